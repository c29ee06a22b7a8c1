// Quality of a layout on a sample of points (thesis, chapter "Quality
// metrics": Sec. "Rank-based criteria", Sec. "Neighbor hit",
// Sec. "Trustworthiness and continuity").  Off the timed path.
//
// Everything is decided by the order of the points around a sample row r:
// all M points (r itself included) sorted by (delta_rl, l) with delta the
// squared Euclidean distance, accumulated in FP64 from the FP32 coordinates
// in dimension order, ties to the lower index.  The rank rho_rj is the
// position of j in that order; the neighbourhood of size k is positions
// 1..k.  FP64 makes these integer decisions the same as a plain FP64
// evaluation of the same definition (each per-dimension term (x - y)^2 of
// two FP32 values is exact in FP64; only the additions round).
//
// eval_scan_kernel: one wavefront per 64 sample rows (one row per lane) and
// one contiguous chunk of the candidates (blockIdx.y).  Candidate tiles are
// staged in LDS as FP64, a chunk of dimensions at a time, and read by all
// lanes at once (broadcast); each lane keeps its row's best k + 1 (distance,
// index) pairs sorted in LDS (neighbour mode) or counts, for each of its kc
// thresholds, the candidates that come before it (rank mode).  A merge
// kernel takes the best k + 1 of the chunks' lists and drops position 0.
#include <cfloat>
#include <climits>
#include <cmath>

#include "ivhd_internal.h"

namespace ivhd {
namespace {

constexpr int kEvalLanes = 64;
constexpr int kEvalTile = 32;       // candidates per tile
constexpr int kEvalDimChunk = 32;   // dimensions staged at a time (2 for 2-D layouts, 8 up to 8-D)

__device__ __forceinline__ bool pair_before(double a, int32_t ia, double b, int32_t ib) {
  return a < b || (a == b && ia < ib);
}

// MODE 0: neighbour lists; MODE 1: rank counts.  Candidates go in tiles of
// kEvalTile; each tile's coordinates are staged in LDS as FP64, DC
// dimensions at a time (read by all lanes at once), while each lane's own
// row chunk sits in registers; every lane keeps the tile's kEvalTile running
// distances in registers, adding dimensions in order, then parks them in
// LDS for the per-candidate pass (list insertion or rank counting).
// Dynamic LDS: the chunk [kEvalTile][DC] doubles, each lane's kEvalTile
// finished distances, then per lane either the list (kl doubles and kl
// ints) or the thresholds and counts (kl doubles, kl ints, kl ints).
template <int MODE, int DC>
__global__ void __launch_bounds__(kEvalLanes)
eval_scan_kernel(const float *__restrict__ Z, int64_t M, int N, const int32_t *__restrict__ rows, int64_t Q, int kl,
                 int64_t chunk, const int32_t *__restrict__ cand, double *__restrict__ part_d,
                 int32_t *__restrict__ part_i, int32_t *__restrict__ rank_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char eval_lds[];
  double *tile = (double *)eval_lds;                        // [kEvalTile][DC]
  double *dist = tile + kEvalTile * DC;                     // [64][kEvalTile]: each lane's tile distances
  double *ld = dist + kEvalLanes * kEvalTile;               // [64][kl]
  int32_t *li = (int32_t *)(ld + (size_t)kEvalLanes * kl);  // [64][kl]
  int32_t *lc = li + (size_t)kEvalLanes * kl;               // rank mode: [64][kl] counts
  const int lane = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * kEvalLanes + lane;
  const bool qvalid = q < Q;
  const int32_t r = qvalid ? rows[q] : 0;
  const float *qrow = Z + (int64_t)r * N;
  double *myd = ld + (size_t)lane * kl;
  int32_t *myi = li + (size_t)lane * kl;
  int32_t *myc = lc + (size_t)lane * kl;
  if (MODE == 0) {
    for (int p = 0; p < kl; ++p) { myd[p] = DBL_MAX; myi[p] = INT32_MAX; }
  } else {
    // thresholds: the distance of each given candidate, in the same order of additions
    for (int c = 0; c < kl; ++c) {
      const int32_t j = qvalid ? cand[q * kl + c] : 0;
      const float *zr = Z + (int64_t)j * N;
      double acc = 0.0;
      for (int n = 0; n < N; ++n) {
        const double t = (double)zr[n] - (qvalid ? (double)qrow[n] : 0.0);
        acc = __dadd_rn(acc, __dmul_rn(t, t));
      }
      myd[c] = acc;
      myi[c] = j;
      myc[c] = 0;
    }
  }
  const int64_t c0 = (int64_t)blockIdx.y * chunk;
  const int64_t c1 = c0 + chunk < M ? c0 + chunk : M;
  for (int64_t t0 = c0; t0 < c1; t0 += kEvalTile) {
    double acc[kEvalTile];
#pragma unroll
    for (int c = 0; c < kEvalTile; ++c) acc[c] = 0.0;
    for (int n0 = 0; n0 < N; n0 += DC) {
      __syncthreads();
      // stage the chunk (rows past c1 and dimensions past N are zero: they add nothing)
      for (int e = lane; e < kEvalTile * DC; e += kEvalLanes) {
        const int c = e / DC, d = e - c * DC;
        const int64_t row = t0 + c;
        tile[e] = (row < c1 && n0 + d < N) ? (double)Z[row * N + n0 + d] : 0.0;
      }
      float qv[DC];
#pragma unroll
      for (int d = 0; d < DC; ++d) qv[d] = (qvalid && n0 + d < N) ? qrow[n0 + d] : 0.f;
      __syncthreads();
#pragma unroll 4
      for (int d = 0; d < DC; ++d) {
        const double qd = (double)qv[d];
#pragma unroll
        for (int c = 0; c < kEvalTile; ++c) {
          const double t = tile[c * DC + d] - qd;
          acc[c] = __dadd_rn(acc[c], __dmul_rn(t, t));
        }
      }
    }
    if (!qvalid) continue;
    double *mydist = dist + lane * kEvalTile;
#pragma unroll
    for (int c = 0; c < kEvalTile; ++c) mydist[c] = acc[c];
    for (int c = 0; c < kEvalTile; ++c) {
      const int64_t l = t0 + c;
      if (l >= c1) break;
      const double d = mydist[c];
      if (MODE == 0) {
        if (pair_before(d, (int32_t)l, myd[kl - 1], myi[kl - 1])) {
          int p = kl - 1;
          while (p > 0 && pair_before(d, (int32_t)l, myd[p - 1], myi[p - 1])) {
            myd[p] = myd[p - 1];
            myi[p] = myi[p - 1];
            --p;
          }
          myd[p] = d;
          myi[p] = (int32_t)l;
        }
      } else {
        for (int e = 0; e < kl; ++e) myc[e] += pair_before(d, (int32_t)l, myd[e], myi[e]) ? 1 : 0;
      }
    }
  }
  if (!qvalid) return;
  if (MODE == 0) {
    const int64_t base = (q * gridDim.y + blockIdx.y) * kl;
    for (int p = 0; p < kl; ++p) {
      part_d[base + p] = myd[p];
      part_i[base + p] = myi[p];
    }
  } else {
    for (int e = 0; e < kl; ++e)
      if (myc[e]) atomicAdd(&rank_out[q * kl + e], myc[e]);
  }
}

// best kl of the S chunk lists of each row, position 0 dropped
__global__ void eval_merge_kernel(const double *__restrict__ part_d, const int32_t *__restrict__ part_i, int64_t Q,
                                  int S, int kl, int32_t *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  int head[64];
  for (int s = 0; s < S; ++s) head[s] = 0;
  const double *D = part_d + q * S * kl;
  const int32_t *I = part_i + q * S * kl;
  for (int p = 0; p < kl; ++p) {
    int best = -1;
    for (int s = 0; s < S; ++s) {
      if (head[s] >= kl) continue;
      const int64_t e = (int64_t)s * kl + head[s];
      if (best < 0 || pair_before(D[e], I[e], D[(int64_t)best * kl + head[best]], I[(int64_t)best * kl + head[best]]))
        best = s;
    }
    const int32_t j = I[(int64_t)best * kl + head[best]];
    head[best] += 1;
    if (p > 0) out[q * (kl - 1) + (p - 1)] = j;
  }
}

// per-row counts of the sample scores, summed with integer atomics (exact,
// order-free): [0] |v ∩ n| over the first k, [1] same-label neighbours in n,
// [2] sum over n \ v of (rank in X - k)
__global__ void eval_scores_kernel(const int32_t *__restrict__ rows, int64_t Q, const int32_t *__restrict__ nx, int kx,
                                   const int32_t *__restrict__ ny, int ky, const int32_t *__restrict__ rank_y,
                                   const int32_t *__restrict__ labels, int k, unsigned long long *__restrict__ sums) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  unsigned long long hits = 0, same = 0, trust = 0;
  const int32_t *vx = nx ? nx + q * kx : nullptr;
  const int32_t *vy = ny + q * ky;
  const int32_t lab = labels ? labels[rows[q]] : 0;
  for (int c = 0; c < k; ++c) {
    const int32_t j = vy[c];
    bool in_x = false;
    if (vx)
      for (int e = 0; e < k; ++e) in_x = in_x || vx[e] == j;
    hits += in_x ? 1 : 0;
    if (labels) same += labels[j] == lab ? 1 : 0;
    if (rank_y && !in_x) trust += (unsigned long long)(rank_y[q * ky + c] - k);
  }
  atomicAdd(&sums[0], hits);
  atomicAdd(&sums[1], same);
  atomicAdd(&sums[2], trust);
}

__global__ void eval_zero_kernel(int32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// chunks of the candidate range: enough blocks to fill the chip, chunks of
// at least 2048 candidates, at most 64 of them
int eval_chunks(int64_t Q, int64_t M) {
  const int64_t qb = (Q + kEvalLanes - 1) / kEvalLanes;
  int64_t S = (2048 + qb - 1) / qb;
  const int64_t smax = M / 2048 > 1 ? M / 2048 : 1;
  if (S > smax) S = smax;
  if (S > 64) S = 64;
  if (S < 1) S = 1;
  return (int)S;
}

template <int MODE, int DC>
hipError_t launch_scan_dc(const float *Z, int64_t M, int N, const int32_t *rows, int64_t Q, int kl, int S,
                          const int32_t *cand, double *part_d, int32_t *part_i, int32_t *rank_out, hipStream_t s) {
  const int64_t chunk = (M + S - 1) / S;
  const dim3 grid((unsigned)((Q + kEvalLanes - 1) / kEvalLanes), (unsigned)S);
  const size_t bytes = (size_t)kEvalTile * DC * 8 + (size_t)kEvalLanes * kEvalTile * 8 +
                       (size_t)kEvalLanes * kl * (MODE == 0 ? 12 : 16);
  hipError_t e = hipFuncSetAttribute((const void *)eval_scan_kernel<MODE, DC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  eval_scan_kernel<MODE, DC><<<grid, kEvalLanes, bytes, s>>>(Z, M, N, rows, Q, kl, chunk, cand, part_d, part_i,
                                                             rank_out);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_scan(const float *Z, int64_t M, int N, const int32_t *rows, int64_t Q, int kl, int S,
                       const int32_t *cand, double *part_d, int32_t *part_i, int32_t *rank_out, hipStream_t s) {
  if (N <= 2) return launch_scan_dc<MODE, 2>(Z, M, N, rows, Q, kl, S, cand, part_d, part_i, rank_out, s);
  if (N <= 8) return launch_scan_dc<MODE, 8>(Z, M, N, rows, Q, kl, S, cand, part_d, part_i, rank_out, s);
  return launch_scan_dc<MODE, kEvalDimChunk>(Z, M, N, rows, Q, kl, S, cand, part_d, part_i, rank_out, s);
}

int eval_max_k() { return 128; }
int eval_max_rank_k() { return 64; }
int eval_max_dims() { return 1024; }

hipError_t launch_eval_neighbours(const float *Z, int64_t M, int N, const int32_t *rows, int64_t Q, int k,
                                  double *part_d, int32_t *part_i, int32_t *out, hipStream_t s) {
  const int S = eval_chunks(Q, M);
  hipError_t e = launch_scan<0>(Z, M, N, rows, Q, k + 1, S, nullptr, part_d, part_i, nullptr, s);
  if (e != hipSuccess) return e;
  eval_merge_kernel<<<grid_for(Q), kBlock, 0, s>>>(part_d, part_i, Q, S, k + 1, out);
  return hipGetLastError();
}

size_t eval_neighbours_scratch(int64_t Q, int64_t M, int k) {
  return (size_t)Q * eval_chunks(Q, M) * (k + 1);
}

hipError_t launch_eval_ranks(const float *Z, int64_t M, int N, const int32_t *rows, int64_t Q, const int32_t *cand,
                             int kc, int32_t *rank_out, hipStream_t s) {
  eval_zero_kernel<<<grid_for(Q * kc), kBlock, 0, s>>>(rank_out, Q * kc);
  return launch_scan<1>(Z, M, N, rows, Q, kc, eval_chunks(Q, M), cand, nullptr, nullptr, rank_out, s);
}

hipError_t launch_eval_scores(const int32_t *rows, int64_t Q, const int32_t *nx, int kx, const int32_t *ny, int ky,
                              const int32_t *rank_y, const int32_t *labels, int k, unsigned long long *sums,
                              hipStream_t s) {
  eval_zero_kernel<<<1, kBlock, 0, s>>>((int32_t *)sums, 6);
  eval_scores_kernel<<<grid_for(Q), kBlock, 0, s>>>(rows, Q, nx, kx, ny, ky, rank_y, labels, k, sums);
  return hipGetLastError();
}

}  // namespace
}  // namespace ivhd

// ---- C ABI ----------------------------------------------------------------
using namespace ivhd;

namespace {

int check_sample(const float *d_z, int64_t M, int32_t N, const int32_t *d_rows, int64_t Q) {
  if (!d_z || (Q > 0 && !d_rows)) return fail(IVHD_EINVAL, "d_z and d_rows must not be NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (N < 1 || N > eval_max_dims()) return fail(IVHD_EINVAL, "N = %d outside [1, %d]", N, eval_max_dims());
  if (Q < 0) return fail(IVHD_EINVAL, "Q = %lld < 0", (long long)Q);
  return IVHD_OK;
}

// device range check of index arrays (entries must lie in [0, hi)); synchronises s
int check_indices(const int32_t *const *arrays, const int64_t *counts, int n, int64_t hi, hipStream_t s) {
  int32_t *flags = nullptr;
  int rc = dev_alloc(&flags, FLAG_SLOTS, "device flags");
  if (rc) return rc;
  hipError_t e = launch_fill_i32(flags, FLAG_SLOTS, 0, s);
  for (int a = 0; a < n && e == hipSuccess; ++a)
    if (arrays[a] && counts[a] > 0) e = launch_range_check(arrays[a], counts[a], (int32_t)hi, flags, s);
  int32_t h[FLAG_SLOTS] = {0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, flags, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flags);
  if (e != hipSuccess) return hip_fail(e, "index range check");
  if (h[FLAG_BAD_INDEX]) return fail(IVHD_EINVAL, "an index entry is outside [0, %lld)", (long long)hi);
  return IVHD_OK;
}

}  // namespace

extern "C" {

int ivhd_eval_neighbours(const float *d_z, int64_t M, int32_t N, const int32_t *d_rows, int64_t Q, int32_t k,
                         int32_t *d_idx, void *stream) {
  clear_error();
  int rc = check_sample(d_z, M, N, d_rows, Q);
  if (rc) return rc;
  if (!d_idx) return fail(IVHD_EINVAL, "d_idx is NULL");
  const int64_t kmax = M - 1 < eval_max_k() ? M - 1 : eval_max_k();
  if (k < 1 || k > kmax) return fail(IVHD_EINVAL, "k = %d outside [1, %lld]", k, (long long)kmax);
  if (Q == 0) return IVHD_OK;
  hipStream_t s = (hipStream_t)stream;
  const int32_t *arrays[] = {d_rows};
  const int64_t counts[] = {Q};
  if ((rc = check_indices(arrays, counts, 1, M, s))) return rc;
  const size_t n = eval_neighbours_scratch(Q, M, k);
  double *part_d = nullptr;
  int32_t *part_i = nullptr;
  if ((rc = dev_alloc(&part_d, n, "chunk lists (distances)"))) return rc;
  if ((rc = dev_alloc(&part_i, n, "chunk lists (indices)"))) {
    (void)hipFree(part_d);
    return rc;
  }
  hipError_t e = launch_eval_neighbours(d_z, M, N, d_rows, Q, k, part_d, part_i, d_idx, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part_d);
  (void)hipFree(part_i);
  if (e != hipSuccess) return hip_fail(e, "eval neighbours");
  return IVHD_OK;
}

int ivhd_eval_ranks(const float *d_z, int64_t M, int32_t N, const int32_t *d_rows, int64_t Q, const int32_t *d_cand,
                    int32_t kc, int32_t *d_rank, void *stream) {
  clear_error();
  int rc = check_sample(d_z, M, N, d_rows, Q);
  if (rc) return rc;
  if (!d_cand || !d_rank) return fail(IVHD_EINVAL, "d_cand and d_rank must not be NULL");
  if (kc < 1 || kc > eval_max_rank_k()) return fail(IVHD_EINVAL, "kc = %d outside [1, %d]", kc, eval_max_rank_k());
  if (Q == 0) return IVHD_OK;
  hipStream_t s = (hipStream_t)stream;
  const int32_t *arrays[] = {d_rows, d_cand};
  const int64_t counts[] = {Q, Q * kc};
  if ((rc = check_indices(arrays, counts, 2, M, s))) return rc;
  hipError_t e = launch_eval_ranks(d_z, M, N, d_rows, Q, d_cand, kc, d_rank, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "eval ranks");
  return IVHD_OK;
}

int ivhd_eval_scores(int64_t M, const int32_t *d_rows, int64_t Q, const int32_t *d_nx, int32_t kx, const int32_t *d_ny,
                     int32_t ky, const int32_t *d_rank_y, const int32_t *d_labels, int32_t k, double *h_out,
                     void *stream) {
  clear_error();
  if (!h_out) return fail(IVHD_EINVAL, "h_out is NULL");
  if (!d_ny || !d_rows) return fail(IVHD_EINVAL, "d_rows and d_ny must not be NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (Q < 1) return fail(IVHD_EINVAL, "Q = %lld < 1", (long long)Q);
  if (k < 1 || k > ky) return fail(IVHD_EINVAL, "k = %d outside [1, ky = %d]", k, ky);
  if (d_nx && k > kx) return fail(IVHD_EINVAL, "k = %d above kx = %d", k, kx);
  if (d_rank_y && !d_nx) return fail(IVHD_EINVAL, "d_rank_y needs d_nx (the ranks count only points outside it)");
  hipStream_t s = (hipStream_t)stream;
  const int32_t *arrays[] = {d_rows, d_ny, d_nx};
  const int64_t counts[] = {Q, Q * ky, d_nx ? Q * kx : 0};
  int rc = check_indices(arrays, counts, 3, M, s);
  if (rc) return rc;
  unsigned long long *sums = nullptr;
  if ((rc = dev_alloc(&sums, 3, "score sums"))) return rc;
  unsigned long long h[3] = {0, 0, 0};
  hipError_t e = launch_eval_scores(d_rows, Q, d_nx, kx, d_ny, ky, d_rank_y, d_labels, k, sums, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(sums);
  if (e != hipSuccess) return hip_fail(e, "eval scores");
  const double kq = (double)k * (double)Q;
  h_out[0] = d_nx ? (double)h[0] / kq : NAN;
  h_out[1] = d_labels ? (double)h[1] / kq : NAN;
  const double den = kq * (2.0 * (double)M - 3.0 * k - 1.0);
  h_out[2] = (d_rank_y && den > 0) ? 1.0 - 2.0 / den * (double)h[2] : NAN;
  return IVHD_OK;
}

}  // extern "C"
