// Exact brute-force k nearest neighbours on gfx950: the input preparation
// of the loop (the thesis builds its kNN graphs with an approximate GPU
// library; here the graph is exact).
//
// Order: squared Euclidean distance, ties to the lower index, the query
// itself excluded.
//
// A block of 256 threads (4 waves) owns 128 queries and sweeps all
// candidates in tiles of 64.  The dot products of a 128 x 64 tile come from
// FP32 MFMA (v_mfma_f32_16x16x4f32), with both operand tiles staged in LDS
// 16 features at a time.  The ranking score |x_c|^2 - 2 q.x_c (|q|^2 is
// the same for the whole row) goes to LDS, where two threads per query row
// keep running top-KP lists in registers.  At the end the two lists are
// merged and the KP survivors are re-ranked by their exact FP32 distance
// sum_k (q_k - x_k)^2, which removes the cancellation error of the
// expanded form; KP >= k + 4 leaves room for candidates the score misranks.
#include <cfloat>

#include "ivhd_internal.h"

namespace ivhd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int QB = 128;        // queries per block
constexpr int CB = 64;         // candidates per tile
constexpr int KC = 16;         // features per staged chunk
constexpr int QP = QB + 16;    // LDS row pitch (== 16 mod 32: the two 16-lane
constexpr int CP = CB + 16;    //   groups of an operand read hit disjoint banks)
constexpr int SP = CB + 1;     // score tile pitch
constexpr int kKnnThreads = 256;

__device__ __forceinline__ bool pair_less(float a, int32_t ia, float b, int32_t ib) {
  return a < b || (a == b && ia < ib);
}

template <int KP>
__device__ __forceinline__ void list_insert(float (&ks)[KP], int32_t (&ki)[KP], float s, int32_t j) {
  if (!pair_less(s, j, ks[KP - 1], ki[KP - 1])) return;
  ks[KP - 1] = s;
  ki[KP - 1] = j;
#pragma unroll
  for (int p = KP - 1; p > 0; --p) {
    if (pair_less(ks[p], ki[p], ks[p - 1], ki[p - 1])) {
      float t = ks[p]; ks[p] = ks[p - 1]; ks[p - 1] = t;
      int32_t u = ki[p]; ki[p] = ki[p - 1]; ki[p - 1] = u;
    }
  }
}

__global__ void __launch_bounds__(256) row_norms_kernel(const float *__restrict__ X, int64_t M, int N,
                                                        float *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= M) return;
  const float *x = X + row * N;
  float s = 0.f;
  for (int k = lane; k < N; k += 64) s += x[k] * x[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[row] = s;
}

// self_mode: 0 = no exclusion, 1 = query q excludes candidate q, 2 = self[q]
template <int KP>
__global__ void __launch_bounds__(kKnnThreads)
knn_kernel(const float *__restrict__ X, int64_t M, int N, const float *__restrict__ Q, int64_t nq,
           int self_mode, const int32_t *__restrict__ self, const float *__restrict__ cnorm, int k,
           int32_t *__restrict__ out_idx, float *__restrict__ out_dist) {
  __shared__ float sQ[KC * QP];
  __shared__ float sC[KC * CP];
  __shared__ float sS[QB * SP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.x * QB;

  // scan ownership: two threads per query row, interleaved columns
  const int my_row = tid >> 1;
  const int half = tid & 1;
  const int64_t my_q = q0 + my_row;
  int64_t my_self = -1;
  if (my_q < nq) my_self = self_mode == 1 ? my_q : (self_mode == 2 ? (int64_t)self[my_q] : -1);

  float ks[KP];
  int32_t ki[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) { ks[p] = FLT_MAX; ki[p] = INT32_MAX; }

  for (int64_t c0 = 0; c0 < M; c0 += CB) {
    floatx4 acc[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int kc = 0; kc < N; kc += KC) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < (QB * KC) / kKnnThreads; ++i) {
        const int e = tid + kKnnThreads * i;
        const int r = e / KC, kk = e % KC;
        const int64_t q = q0 + r;
        float v = 0.f;
        if (q < nq && kc + kk < N) v = Q[q * N + kc + kk];
        sQ[kk * QP + r] = v;
      }
#pragma unroll
      for (int i = 0; i < (CB * KC) / kKnnThreads; ++i) {
        const int e = tid + kKnnThreads * i;
        const int r = e / KC, kk = e % KC;
        const int64_t c = c0 + r;
        float v = 0.f;
        if (c < M && kc + kk < N) v = X[c * N + kc + kk];
        sC[kk * CP + r] = v;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < KC / 4; ++s) {
        const int kidx = 4 * s + (lane >> 4);
        float a[2], b[4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) a[rb] = sQ[kidx * QP + 32 * wave + 16 * rb + (lane & 15)];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) b[cb] = sC[kidx * CP + 16 * cb + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
      }
    }

    // scores into LDS: D[i][j] of a 16x16 block sits in lane j + 16*(i/4), register i%4
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = 16 * cb + (lane & 15);
      const int64_t c = c0 + col;
      const float cn = c < M ? cnorm[c] : 0.f;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 32 * wave + 16 * rb + 4 * (lane >> 4) + r;
          sS[row * SP + col] = cn - 2.f * acc[rb][cb][r];
        }
    }
    __syncthreads();
    if (my_q < nq) {
      for (int m = 0; m < CB / 2; ++m) {
        const int col = 2 * m + half;
        const int64_t c = c0 + col;
        if (c >= M || c == my_self) continue;
        list_insert<KP>(ks, ki, sS[my_row * SP + col], (int32_t)c);
      }
    }
  }

  // merge the two lists of each row (through LDS), then re-rank exactly
  __syncthreads();
  float *mS = sS;                                // [QB][KP] scores
  int32_t *mI = (int32_t *)(sS + QB * KP);       // [QB][KP] indices
  if (half == 1) {
#pragma unroll
    for (int p = 0; p < KP; ++p) { mS[my_row * KP + p] = ks[p]; mI[my_row * KP + p] = ki[p]; }
  }
  __syncthreads();
  if (half == 0 && my_q < nq) {
#pragma unroll
    for (int p = 0; p < KP; ++p) list_insert<KP>(ks, ki, mS[my_row * KP + p], mI[my_row * KP + p]);
    const float *qrow = Q + my_q * N;
    float ed[KP];
#pragma unroll
    for (int p = 0; p < KP; ++p) {
      float d = FLT_MAX;
      if (ki[p] != INT32_MAX) {
        const float *xr = X + (int64_t)ki[p] * N;
        d = 0.f;
        for (int kk = 0; kk < N; ++kk) {
          const float t = qrow[kk] - xr[kk];
          d += t * t;
        }
      }
      ed[p] = d;
    }
    // exact re-rank: insertion sort of (ed, ki), fully unrolled
#pragma unroll
    for (int p = 1; p < KP; ++p) {
#pragma unroll
      for (int q = p; q > 0; --q) {
        if (pair_less(ed[q], ki[q], ed[q - 1], ki[q - 1])) {
          float t = ed[q]; ed[q] = ed[q - 1]; ed[q - 1] = t;
          int32_t u = ki[q]; ki[q] = ki[q - 1]; ki[q - 1] = u;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < KP; ++p) {
      if (p < k) {
        out_idx[my_q * k + p] = ki[p] == INT32_MAX ? -1 : ki[p];
        if (out_dist) out_dist[my_q * k + p] = ed[p];
      }
    }
  }
}

template <int KP>
hipError_t launch_knn_kp(const float *X, int64_t M, int N, const float *Q, int64_t nq, int self_mode,
                         const int32_t *self, const float *cnorm, int k, int32_t *idx, float *dist,
                         hipStream_t s) {
  static_assert(2 * QB * KP <= QB * SP, "merge buffers must fit in the score tile");
  const unsigned grid = (unsigned)((nq + QB - 1) / QB);
  knn_kernel<KP><<<grid, kKnnThreads, 0, s>>>(X, M, N, Q, nq, self_mode, self, cnorm, k, idx, dist);
  return hipGetLastError();
}

}  // namespace

int knn_max_k() { return 28; }

hipError_t launch_row_norms(const float *X, int64_t M, int N, float *out, hipStream_t s) {
  row_norms_kernel<<<grid_for(M, 4), 256, 0, s>>>(X, M, N, out);
  return hipGetLastError();
}

hipError_t launch_knn(const float *X, int64_t M, int N, const float *Q, int64_t nq, int self_mode,
                      const int32_t *self, const float *cnorm, int k, int32_t *idx, float *dist,
                      hipStream_t s) {
  if (k + 4 <= 8) return launch_knn_kp<8>(X, M, N, Q, nq, self_mode, self, cnorm, k, idx, dist, s);
  if (k + 4 <= 16) return launch_knn_kp<16>(X, M, N, Q, nq, self_mode, self, cnorm, k, idx, dist, s);
  return launch_knn_kp<32>(X, M, N, Q, nq, self_mode, self, cnorm, k, idx, dist, s);
}

}  // namespace ivhd
