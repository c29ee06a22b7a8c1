// Exact brute-force k nearest neighbours on gfx950: the input preparation
// of the loop (the thesis builds its kNN graphs with an approximate GPU
// library; here the graph is exact).
//
// Order: squared Euclidean distance, ties to the lower index, the query
// itself excluded.
//
// Dot products on the FP16 matrix cores with FP32 accumulation, at close to
// FP32 accuracy: every coordinate, scaled by a power of two so the largest
// magnitude sits below 2^14, is split into hi = fp16(x) and
// lo = fp16(x - hi) (22 significant bits together), and
//     q.x ~= hi_q.hi_x + hi_q.lo_x + lo_q.hi_x
// (the dropped lo.lo term is below 2^-22 of |q_k x_k|; each fp16 product is
// exact in FP32).  Three v_mfma_f32_16x16x32_f16 per product block give
// about 5x the throughput of the FP32 matrix path.
//
// A block of 256 threads (4 waves) owns 128 queries and sweeps all
// candidates: for padded widths up to 128 in tiles of 64 with the queries'
// operands held in registers (knn_small_kernel), above that in tiles of 128,
// K in steps of 32 staged in LDS (knn_kernel); K is contiguous per LDS row,
// so one lane's operand, 8 consecutive k, is one 16-byte read.  The
// ranking score |x_c|^2 - 2 q.x_c (|q|^2 is the same for the whole row) goes
// to an LDS score tile, where two threads per query row keep running top-KP
// lists in registers.  At the end
// the two lists are merged and the KP survivors are re-ranked by their exact
// FP32 distance sum_k (q_k - x_k)^2, which removes the cancellation error of
// the expanded form; KP >= k + 4 leaves room for candidates the score
// misranks.
#include <cfloat>

#include "ivhd_internal.h"

namespace ivhd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int QB = 128;        // queries per block
constexpr int CB = 64;         // candidates per tile
constexpr int TKK = 32;        // features per staged step
constexpr int HP = TKK + 8;    // LDS row pitch in halves (80 bytes, 16-byte aligned rows)
constexpr int SP = CB + 4;     // score tile pitch (floats; rows 16-byte aligned)
constexpr int kKnnThreads = 256;
constexpr int kSplitMaxExp = 14;   // scaled magnitudes stay below 2^14

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

// largest |x| (as the bits of a non-negative float, so integer max is float
// max); NaN sets the top bits and is reported by the host
__global__ void __launch_bounds__(256) absmax_kernel(const float *__restrict__ X, int64_t n, uint32_t *out) {
  uint32_t m = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = __float_as_uint(X[e]) & 0x7fffffffu;
    m = u > m ? u : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t t = __shfl_xor(m, o, 64);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// hi / lo FP16 rows of scale * X, padded with zeros to Np (a multiple of TKK)
__global__ void split_kernel(const float *__restrict__ X, int64_t M, int N, int Np, float scale,
                             _Float16 *__restrict__ hi, _Float16 *__restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * Np) return;
  const int64_t r = e / Np;
  const int c = (int)(e % Np);
  const float x = c < N ? X[r * N + c] * scale : 0.f;
  const _Float16 h = (_Float16)x;
  hi[e] = h;
  lo[e] = (_Float16)(x - (float)h);
}

// Ranks the CW scores of one thread's half row (sS row `row`, candidates
// cbase..cbase+CW-1, in order) into its list.  A group of four whose
// smallest score lies above the list's last entry is passed over at once:
// none of them could enter the list, so the list ends as if each had been
// offered.  (Lists of 32 keep a one-by-one scan of alternate columns: the
// group test costs registers they do not have.)
template <int KP, int CW>
__device__ __forceinline__ void scan_half_row(const float *__restrict__ row, int64_t cbase, int64_t M,
                                              int64_t my_self, float (&ks)[KP], int32_t (&ki)[KP]) {
#pragma unroll 1
  for (int m = 0; m < CW; m += 4) {
    floatx4 v = *reinterpret_cast<const floatx4 *>(row + m);
    const float lo = fminf(fminf(v.x, v.y), fminf(v.z, v.w));
    if (lo > ks[KP - 1]) continue;
#pragma unroll 1
    for (int e = 0; e < 4; ++e) {   // one insertion body, the group rotated through it
      const float se = v.x;
      v = v.yzwx;
      const int64_t c = cbase + m + e;
      if (c >= M || c == my_self) continue;
      list_insert<KP>(ks, ki, se, (int32_t)c);
    }
  }
}

// Exact FP32 squared distances of a block's (row, survivor) pairs: mI
// [QB][KP] holds the survivors' ids (INT32_MAX: none), mS receives the
// distances; the pairs are spread over the whole block, the features taken in
// order with 16-byte loads where the rows allow.  qrow_of(r) is the query
// row of block row r.
template <int KP, typename QRowOf>
__device__ __forceinline__ void rerank_pairs(float *__restrict__ mS, const int32_t *__restrict__ mI,
                                             const float *__restrict__ Q, const float *__restrict__ X, int N,
                                             QRowOf qrow_of) {
  const bool vec4 = N % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
#pragma unroll 1
  for (int t = threadIdx.x; t < QB * KP; t += kKnnThreads) {
    const int32_t id = mI[t];
    float d = FLT_MAX;
    if (id != INT32_MAX) {
      const float *qr = Q + qrow_of(t / KP) * N, *xr = X + (int64_t)id * N;
      d = 0.f;
      if (vec4) {
        for (int kk = 0; kk < N; kk += 4) {
          const float4 u = *reinterpret_cast<const float4 *>(qr + kk);
          const float4 v = *reinterpret_cast<const float4 *>(xr + kk);
          float e = u.x - v.x;
          d += e * e;
          e = u.y - v.y;
          d += e * e;
          e = u.z - v.z;
          d += e * e;
          e = u.w - v.w;
          d += e * e;
        }
      } else {
        for (int kk = 0; kk < N; ++kk) {
          const float e = qr[kk] - xr[kk];
          d += e * e;
        }
      }
    }
    mS[t] = d;
  }
}

// a row's KP (distance, id) pairs sorted in place, ascending
template <int KP>
__device__ __forceinline__ void sort_row(float *__restrict__ rs, int32_t *__restrict__ ri) {
#pragma unroll 1
  for (int p = 1; p < KP; ++p) {
    const float dv = rs[p];
    const int32_t iv = ri[p];
    int q = p;
    while (q > 0 && pair_less(dv, iv, rs[q - 1], ri[q - 1])) {
      rs[q] = rs[q - 1];
      ri[q] = ri[q - 1];
      --q;
    }
    rs[q] = dv;
    ri[q] = iv;
  }
}

// End of a query block: the two running lists of each row are merged
// (through LDS, sS holding at least 2 QB KP words), the survivors are
// re-ranked by their exact FP32 distances (the whole block computing them)
// and the best k written out.
template <int KP>
__device__ __forceinline__ void finish_rows(float *sS, float (&ks)[KP], int32_t (&ki)[KP], int my_row, int half,
                                            int64_t my_q, int64_t nq, const float *__restrict__ Q,
                                            const float *__restrict__ X, int N, int k,
                                            int32_t *__restrict__ out_idx, float *__restrict__ out_dist) {
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
  }
  __syncthreads();   // the other half's list has been read
  if (half == 0) {
#pragma unroll
    for (int p = 0; p < KP; ++p) mI[my_row * KP + p] = my_q < nq ? ki[p] : INT32_MAX;
  }
  __syncthreads();
  const int64_t q0 = my_q - my_row;
  rerank_pairs<KP>(mS, mI, Q, X, N, [&](int r) { return q0 + r; });
  __syncthreads();
  if (half == 0 && my_q < nq) {
    float *rs = mS + my_row * KP;
    int32_t *ri = mI + my_row * KP;
    sort_row<KP>(rs, ri);
#pragma unroll 1
    for (int p = 0; p < k; ++p) {
      out_idx[my_q * k + p] = ri[p] == INT32_MAX ? -1 : ri[p];
      if (out_dist) out_dist[my_q * k + p] = rs[p];
    }
  }
}

// Wide data: a block owns 128 queries and sweeps the candidates in tiles of
// CBW = 128; wave (wq, wc) computes the 64 x 64 quarter rows 64 wq.., columns
// 64 wc.. of each tile, so every staged operand byte feeds twice the MFMAs
// of a 64-candidate tile.  The operand rows of K step s + 1 are loaded into
// registers during the MFMAs of step s.
constexpr int CBW = 128;        // candidates per tile (wide kernel)
constexpr int SPW = CBW + 4;    // its score tile pitch (floats; rows 16-byte aligned)

struct WideFrag {
  halfx8 qh[2], ql[2], ch[2], cl[2];   // 128 query and 128 candidate rows x 8 features per thread
};

__device__ __forceinline__ void load_wide(WideFrag &F, const _Float16 *__restrict__ Qh,
                                          const _Float16 *__restrict__ Ql, int64_t nq, int64_t q0,
                                          const _Float16 *__restrict__ Xh, const _Float16 *__restrict__ Xl,
                                          int64_t M, int64_t c0, int Np, int k0) {
  const int kc = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int r = (threadIdx.x + kKnnThreads * c) >> 2;
    const bool okq = q0 + r < nq, okc = c0 + r < M;
    F.qh[c] = okq ? *reinterpret_cast<const halfx8 *>(Qh + (q0 + r) * Np + k0 + kc) : halfx8{};
    F.ql[c] = okq ? *reinterpret_cast<const halfx8 *>(Ql + (q0 + r) * Np + k0 + kc) : halfx8{};
    F.ch[c] = okc ? *reinterpret_cast<const halfx8 *>(Xh + (c0 + r) * Np + k0 + kc) : halfx8{};
    F.cl[c] = okc ? *reinterpret_cast<const halfx8 *>(Xl + (c0 + r) * Np + k0 + kc) : halfx8{};
  }
}

__device__ __forceinline__ void store_wide(const WideFrag &F, _Float16 *sQh, _Float16 *sQl, _Float16 *sCh,
                                           _Float16 *sCl) {
  const int kc = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int r = (threadIdx.x + kKnnThreads * c) >> 2;
    *reinterpret_cast<halfx8 *>(sQh + r * HP + kc) = F.qh[c];
    *reinterpret_cast<halfx8 *>(sQl + r * HP + kc) = F.ql[c];
    *reinterpret_cast<halfx8 *>(sCh + r * HP + kc) = F.ch[c];
    *reinterpret_cast<halfx8 *>(sCl + r * HP + kc) = F.cl[c];
  }
}

// self_mode: 0 = no exclusion, 1 = query q excludes candidate q, 2 = self[q]
template <int KP>
__global__ void __launch_bounds__(kKnnThreads, 2)
knn_kernel(const float *__restrict__ X, int64_t M, int N, const float *__restrict__ Q, int64_t nq,
           const _Float16 *__restrict__ Xh, const _Float16 *__restrict__ Xl, const _Float16 *__restrict__ Qh,
           const _Float16 *__restrict__ Ql, int Np, float inv_scale2, int self_mode,
           const int32_t *__restrict__ self, const float *__restrict__ cnorm, int k,
           int32_t *__restrict__ out_idx, float *__restrict__ out_dist) {
  // one LDS area: the operand tiles during the K loop, then the score tile
  __shared__ __attribute__((aligned(16))) float smem[QB * SPW];
  static_assert((2 * QB + 2 * CBW) * HP * 2 <= QB * SPW * 4, "operand tiles must fit in the score tile");
  static_assert(2 * QB * 32 <= QB * SPW, "merge buffers must fit in the score tile");
  _Float16 *sQh = reinterpret_cast<_Float16 *>(smem);
  _Float16 *sQl = sQh + QB * HP;
  _Float16 *sCh = sQl + QB * HP;
  _Float16 *sCl = sCh + CBW * HP;
  float *sS = smem;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wq = 64 * (wave >> 1), wc = 64 * (wave & 1);
  const int64_t q0 = (int64_t)blockIdx.x * QB;

  // scan ownership: two threads per query row (halves of the columns, or
  // alternate columns for 32-entry lists)
  const int my_row = tid >> 1;
  const int half = tid & 1;
  const int64_t my_q = q0 + my_row;
  int64_t my_self = -1;
  if (my_q < nq) my_self = self_mode == 1 ? my_q : (self_mode == 2 ? (int64_t)self[my_q] : -1);

  float ks[KP];
  int32_t ki[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) { ks[p] = FLT_MAX; ki[p] = INT32_MAX; }

  const int kq = (lane >> 4) * 8;
  static_assert(QB * (TKK / 8) == 2 * kKnnThreads && CBW * (TKK / 8) == 2 * kKnnThreads, "fragment shape");
  WideFrag F;
  load_wide(F, Qh, Ql, nq, q0, Xh, Xl, M, 0, Np, 0);
  for (int64_t c0 = 0; c0 < M; c0 += CBW) {
    floatx4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < Np; k0 += TKK) {
      __syncthreads();   // the previous step's operands, or the previous tile's scores, are consumed
      store_wide(F, sQh, sQl, sCh, sCl);
      __syncthreads();
      {  // prefetch the next step: the next K slice, or the first of the next tile
        int64_t nc0 = c0;
        int nk0 = k0 + TKK;
        if (nk0 >= Np) {
          nk0 = 0;
          nc0 = c0 + CBW;
        }
        if (nc0 < M) load_wide(F, Qh, Ql, nq, q0, Xh, Xl, M, nc0, Np, nk0);
      }
      halfx8 ah[4], al[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int r = wq + 16 * rb + (lane & 15);
        ah[rb] = *reinterpret_cast<const halfx8 *>(sQh + r * HP + kq);
        al[rb] = *reinterpret_cast<const halfx8 *>(sQl + r * HP + kq);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int r = wc + 16 * cb + (lane & 15);
        const halfx8 bh = *reinterpret_cast<const halfx8 *>(sCh + r * HP + kq);
        const halfx8 bl = *reinterpret_cast<const halfx8 *>(sCl + r * HP + kq);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bh, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bl, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[rb], bh, acc[rb][cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();   // operands dead: the area becomes the score tile

    // scores: D[i][j] of a 16x16 block sits in lane j + 16 (i / 4), register i % 4
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = wc + 16 * cb + (lane & 15);
      const int64_t c = c0 + col;
      const float cn = c < M ? cnorm[c] : 0.f;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wq + 16 * rb + 4 * (lane >> 4) + r;
          sS[row * SPW + col] = cn - 2.f * (acc[rb][cb][r] * inv_scale2);
        }
    }
    __syncthreads();
    if (my_q < nq) {
      if constexpr (KP >= 32) {
        for (int m = 0; m < CBW / 2; ++m) {
          const int col = 2 * m + half;
          const int64_t c = c0 + col;
          if (c >= M || c == my_self) continue;
          list_insert<KP>(ks, ki, sS[my_row * SPW + col], (int32_t)c);
        }
      } else
        scan_half_row<KP, CBW / 2>(sS + my_row * SPW + half * (CBW / 2), c0 + half * (CBW / 2), M, my_self, ks,
                                   ki);
    }
  }
  finish_rows<KP>(sS, ks, ki, my_row, half, my_q, nq, Q, X, N, k, out_idx, out_dist);
}

// Narrow data (padded width Np = 32 NS <= 128): each wave keeps its 32
// query rows' hi / lo fragments for all NS K steps in registers for the whole
// sweep, so only the candidate tile is staged, once per tile: its rows for
// the next tile are loaded into registers while this tile is multiplied and
// ranked, and a tile costs two barriers instead of two per K step.  Same
// MFMA sequence per score (K steps in order, hi.hi, hi.lo, lo.hi), so the
// scores, and the answers, are those of knn_kernel.
constexpr int kSmallPitch = 4 * TKK + 8;   // candidate tile pitch in halves (NS <= 4)

template <int KP, int NS>
__global__ void __launch_bounds__(kKnnThreads, 2)
knn_small_kernel(const float *__restrict__ X, int64_t M, int N, const float *__restrict__ Q, int64_t nq,
                 const _Float16 *__restrict__ Xh, const _Float16 *__restrict__ Xl,
                 const _Float16 *__restrict__ Qh, const _Float16 *__restrict__ Ql, float inv_scale2,
                 int self_mode, const int32_t *__restrict__ self, const float *__restrict__ cnorm, int k,
                 int32_t *__restrict__ out_idx, float *__restrict__ out_dist) {
  constexpr int Np = NS * TKK;
  __shared__ __attribute__((aligned(16))) float sS[QB * SP];
  __shared__ __attribute__((aligned(16))) _Float16 sCh[CB * kSmallPitch];
  __shared__ __attribute__((aligned(16))) _Float16 sCl[CB * kSmallPitch];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.x * QB;
  const int my_row = tid >> 1;
  const int half = tid & 1;
  const int64_t my_q = q0 + my_row;
  int64_t my_self = -1;
  if (my_q < nq) my_self = self_mode == 1 ? my_q : (self_mode == 2 ? (int64_t)self[my_q] : -1);

  float ks[KP];
  int32_t ki[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) { ks[p] = FLT_MAX; ki[p] = INT32_MAX; }

  const int kq = (lane >> 4) * 8;
  // this wave's query operands: rows 32 wave + 16 rb + lane % 16
  halfx8 ah[NS][2], al[NS][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const int64_t q = q0 + 32 * wave + 16 * rb + (lane & 15);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      ah[t][rb] = q < nq ? *reinterpret_cast<const halfx8 *>(Qh + q * Np + TKK * t + kq) : halfx8{};
      al[t][rb] = q < nq ? *reinterpret_cast<const halfx8 *>(Ql + q * Np + TKK * t + kq) : halfx8{};
    }
  }
  // candidate rows: thread holds row tid / 4, features 8 (tid % 4) + 32 t
  const int cr = tid >> 2, ckc = (tid & 3) * 8;
  halfx8 ch[NS], cl[NS];
  auto load_cand = [&](int64_t c0) {
    const bool ok = c0 + cr < M;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      ch[t] = ok ? *reinterpret_cast<const halfx8 *>(Xh + (c0 + cr) * Np + TKK * t + ckc) : halfx8{};
      cl[t] = ok ? *reinterpret_cast<const halfx8 *>(Xl + (c0 + cr) * Np + TKK * t + ckc) : halfx8{};
    }
  };
  load_cand(0);
  for (int64_t c0 = 0; c0 < M; c0 += CB) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      *reinterpret_cast<halfx8 *>(sCh + cr * kSmallPitch + TKK * t + ckc) = ch[t];
      *reinterpret_cast<halfx8 *>(sCl + cr * kSmallPitch + TKK * t + ckc) = cl[t];
    }
    __syncthreads();   // tile staged; every thread has finished ranking the previous tile
    if (c0 + CB < M) load_cand(c0 + CB);
    floatx4 acc[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      halfx8 bh[4], bl[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int r = 16 * cb + (lane & 15);
        bh[cb] = *reinterpret_cast<const halfx8 *>(sCh + r * kSmallPitch + TKK * t + kq);
        bl[cb] = *reinterpret_cast<const halfx8 *>(sCl + r * kSmallPitch + TKK * t + kq);
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t][rb], bh[cb], acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t][rb], bl[cb], acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[t][rb], bh[cb], acc[rb][cb], 0, 0, 0);
        }
    }
    // scores: D[i][j] of a 16x16 block sits in lane j + 16 (i / 4), register i % 4
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
          sS[row * SP + col] = cn - 2.f * (acc[rb][cb][r] * inv_scale2);
        }
    }
    __syncthreads();   // scores complete; every wave has finished reading the candidate tile
    if (my_q < nq) {
      if constexpr (KP >= 32) {
        for (int m = 0; m < CB / 2; ++m) {
          const int col = 2 * m + half;
          const int64_t c = c0 + col;
          if (c >= M || c == my_self) continue;
          list_insert<KP>(ks, ki, sS[my_row * SP + col], (int32_t)c);
        }
      } else
        scan_half_row<KP, CB / 2>(sS + my_row * SP + half * (CB / 2), c0 + half * (CB / 2), M, my_self, ks, ki);
    }
  }
  finish_rows<KP>(sS, ks, ki, my_row, half, my_q, nq, Q, X, N, k, out_idx, out_dist);
}

// ---- inverted-file (approximate) search ------------------------------------
// The index: nlist centroids and the points' list assignment.  The points are
// reordered by list (sorted position p holds point pos_id[p]; list c is
// positions [lptr[c], lptr[c+1])), split into hi / lo FP16 rows in that
// order.  The work is list-major: each block takes up to 128 of the queries
// that probe one list (query ids pq[qbeg..qend)) and sweeps that list's
// points with the same MFMA tiles, score tile and top-KP lists as the exact
// kernel, then re-ranks its survivors exactly and writes them to the query's
// probe slot.  A merge kernel then takes each query's best k over its slots.

__global__ void gather_f32_kernel(const float *__restrict__ src, const int32_t *__restrict__ idx, int64_t n,
                                  float *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[idx[e]];
}

// rows of the split arrays in list order
__global__ void split_gather_kernel(const float *__restrict__ X, int64_t M, int N, int Np, float scale,
                                    const int32_t *__restrict__ pos_id, _Float16 *__restrict__ hi,
                                    _Float16 *__restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * Np) return;
  const int64_t p = e / Np;
  const int c = (int)(e % Np);
  const float x = c < N ? X[(int64_t)pos_id[p] * N + c] * scale : 0.f;
  const _Float16 h = (_Float16)x;
  hi[e] = h;
  lo[e] = (_Float16)(x - (float)h);
}

// one K step of the list kernel's operands in registers (loaded a step ahead):
// 128 query rows (ids pq[qbeg + r] while qbeg + r < qend) and 128 contiguous
// list rows c0 + r while < pend, 8 features per chunk
struct IvfFrag {
  halfx8 qh[2], ql[2], ch[2], cl[2];
};

__device__ __forceinline__ void load_ivf(IvfFrag &F, const _Float16 *__restrict__ Qh,
                                         const _Float16 *__restrict__ Ql, const int32_t *__restrict__ pq,
                                         int64_t qbeg, int64_t qend, const _Float16 *__restrict__ Xh,
                                         const _Float16 *__restrict__ Xl, int64_t c0, int64_t pend, int Np, int k0) {
  const int kc = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int r = (threadIdx.x + kKnnThreads * c) >> 2;
    const bool ok = qbeg + r < qend;
    const int64_t row = ok ? (int64_t)pq[qbeg + r] : 0;
    F.qh[c] = ok ? *reinterpret_cast<const halfx8 *>(Qh + row * Np + k0 + kc) : halfx8{};
    F.ql[c] = ok ? *reinterpret_cast<const halfx8 *>(Ql + row * Np + k0 + kc) : halfx8{};
    const bool okc = c0 + r < pend;
    F.ch[c] = okc ? *reinterpret_cast<const halfx8 *>(Xh + (c0 + r) * Np + k0 + kc) : halfx8{};
    F.cl[c] = okc ? *reinterpret_cast<const halfx8 *>(Xl + (c0 + r) * Np + k0 + kc) : halfx8{};
  }
}

__device__ __forceinline__ void store_ivf(const IvfFrag &F, _Float16 *sQh, _Float16 *sQl, _Float16 *sCh,
                                          _Float16 *sCl) {
  const int kc = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int r = (threadIdx.x + kKnnThreads * c) >> 2;
    *reinterpret_cast<halfx8 *>(sQh + r * HP + kc) = F.qh[c];
    *reinterpret_cast<halfx8 *>(sQl + r * HP + kc) = F.ql[c];
    *reinterpret_cast<halfx8 *>(sCh + r * HP + kc) = F.ch[c];
    *reinterpret_cast<halfx8 *>(sCl + r * HP + kc) = F.cl[c];
  }
}

// the list kernel tiles like knn_kernel: 128 queries x 128 list points per
// tile, each wave a 64 x 64 quarter
template <int KP>
__global__ void __launch_bounds__(kKnnThreads, 2)
ivf_list_kernel(const float *__restrict__ X, int N, const float *__restrict__ Q, const _Float16 *__restrict__ Xh,
                const _Float16 *__restrict__ Xl, const _Float16 *__restrict__ Qh, const _Float16 *__restrict__ Ql,
                int Np, float inv_scale2, const float *__restrict__ pnorm, const int32_t *__restrict__ pos_id,
                const int32_t *__restrict__ lptr, const int32_t *__restrict__ pptr, const int32_t *__restrict__ pq,
                const int32_t *__restrict__ work_list, const int32_t *__restrict__ work_chunk,
                const int32_t *__restrict__ probes, int nprobe, const int32_t *__restrict__ self, int k,
                int32_t *__restrict__ part_idx, float *__restrict__ part_dist) {
  __shared__ __attribute__((aligned(16))) float smem[QB * SPW];
  static_assert((2 * QB + 2 * CBW) * HP * 2 <= QB * SPW * 4, "operand tiles must fit in the score tile");
  _Float16 *sQh = reinterpret_cast<_Float16 *>(smem);
  _Float16 *sQl = sQh + QB * HP;
  _Float16 *sCh = sQl + QB * HP;
  _Float16 *sCl = sCh + CBW * HP;
  float *sS = smem;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wq = 64 * (wave >> 1), wc = 64 * (wave & 1);
  const int32_t c = work_list[blockIdx.x];
  const int64_t qbeg = (int64_t)pptr[c] + (int64_t)work_chunk[blockIdx.x] * QB;
  const int64_t qend = pptr[c + 1];
  const int64_t pbeg = lptr[c], pend = lptr[c + 1];

  const int my_row = tid >> 1;
  const int half = tid & 1;
  const bool have_q = qbeg + my_row < qend;
  const int32_t my_q = have_q ? pq[qbeg + my_row] : -1;
  const int32_t my_self = have_q && self ? self[my_q] : -1;

  float ks[KP];
  int32_t ki[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) { ks[p] = FLT_MAX; ki[p] = INT32_MAX; }

  const int kq = (lane >> 4) * 8;
  static_assert(QB * (TKK / 8) == 2 * kKnnThreads && CBW * (TKK / 8) == 2 * kKnnThreads, "fragment shape");
  IvfFrag F;
  if (pbeg < pend) load_ivf(F, Qh, Ql, pq, qbeg, qend, Xh, Xl, pbeg, pend, Np, 0);
  for (int64_t c0 = pbeg; c0 < pend; c0 += CBW) {
    floatx4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Np; k0 += TKK) {
      __syncthreads();   // the previous step's operands, or the previous tile's scores, are consumed
      store_ivf(F, sQh, sQl, sCh, sCl);
      __syncthreads();
      {  // prefetch the next K slice, or the first of the next tile
        int64_t nc0 = c0;
        int nk0 = k0 + TKK;
        if (nk0 >= Np) {
          nk0 = 0;
          nc0 = c0 + CBW;
        }
        if (nc0 < pend) load_ivf(F, Qh, Ql, pq, qbeg, qend, Xh, Xl, nc0, pend, Np, nk0);
      }
      halfx8 ah[4], al[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int r = wq + 16 * rb + (lane & 15);
        ah[rb] = *reinterpret_cast<const halfx8 *>(sQh + r * HP + kq);
        al[rb] = *reinterpret_cast<const halfx8 *>(sQl + r * HP + kq);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int r = wc + 16 * cb + (lane & 15);
        const halfx8 bh = *reinterpret_cast<const halfx8 *>(sCh + r * HP + kq);
        const halfx8 bl = *reinterpret_cast<const halfx8 *>(sCl + r * HP + kq);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bh, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bl, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[rb], bh, acc[rb][cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = wc + 16 * cb + (lane & 15);
      const float cn = c0 + col < pend ? pnorm[c0 + col] : 0.f;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wq + 16 * rb + 4 * (lane >> 4) + r;
          sS[row * SPW + col] = cn - 2.f * (acc[rb][cb][r] * inv_scale2);
        }
    }
    __syncthreads();
    if (have_q) {
      for (int m = 0; m < CBW / 2; ++m) {
        const int col = 2 * m + half;
        if (c0 + col >= pend) continue;
        const int32_t id = pos_id[c0 + col];
        if (id == my_self) continue;
        list_insert<KP>(ks, ki, sS[my_row * SPW + col], id);
      }
    }
  }

  __syncthreads();
  float *mS = sS;
  int32_t *mI = (int32_t *)(sS + QB * KP);
  if (half == 1) {
#pragma unroll
    for (int p = 0; p < KP; ++p) { mS[my_row * KP + p] = ks[p]; mI[my_row * KP + p] = ki[p]; }
  }
  __syncthreads();
  if (half == 0 && have_q) {
#pragma unroll
    for (int p = 0; p < KP; ++p) list_insert<KP>(ks, ki, mS[my_row * KP + p], mI[my_row * KP + p]);
  }
  __syncthreads();   // the other half's list has been read
  if (half == 0) {
#pragma unroll
    for (int p = 0; p < KP; ++p) mI[my_row * KP + p] = have_q ? ki[p] : INT32_MAX;
  }
  __syncthreads();
  // exact FP32 distances of every row's survivors over the whole block (a
  // list holds few points, so this is a large share of the work)
  rerank_pairs<KP>(mS, mI, Q, X, N, [&](int r) { return (int64_t)pq[qbeg + r]; });
  __syncthreads();
  if (half == 0 && have_q) {
    float *rs = mS + my_row * KP;
    int32_t *ri = mI + my_row * KP;
    sort_row<KP>(rs, ri);
    // this list's probe slot of the query
    int slot = 0;
    for (int p = 0; p < nprobe; ++p)
      if (probes[(int64_t)my_q * nprobe + p] == c) slot = p;
    int32_t *oi = part_idx + ((int64_t)my_q * nprobe + slot) * k;
    float *od = part_dist + ((int64_t)my_q * nprobe + slot) * k;
#pragma unroll 1
    for (int p = 0; p < k; ++p) {
      oi[p] = ri[p] == INT32_MAX ? -1 : ri[p];
      od[p] = ri[p] == INT32_MAX ? FLT_MAX : rs[p];
    }
  }
}

// each query's k best over its nprobe sorted slots (slots of lists it did not
// probe twice stay at -1 / FLT_MAX from the fill)
__global__ void ivf_merge_kernel(const int32_t *__restrict__ part_idx, const float *__restrict__ part_dist,
                                 int64_t nq, int nprobe, int k, int32_t *__restrict__ out_idx,
                                 float *__restrict__ out_dist) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int head[32];
  for (int p = 0; p < nprobe; ++p) head[p] = 0;
  const int32_t *pi = part_idx + q * nprobe * k;
  const float *pd = part_dist + q * nprobe * k;
  for (int r = 0; r < k; ++r) {
    int best = -1;
    float bd = FLT_MAX;
    int32_t bi = INT32_MAX;
    for (int p = 0; p < nprobe; ++p) {
      if (head[p] >= k) continue;
      const int32_t i = pi[p * k + head[p]];
      if (i < 0) continue;
      const float d = pd[p * k + head[p]];
      if (pair_less(d, i, bd, bi)) { bd = d; bi = i; best = p; }
    }
    if (best >= 0) head[best] += 1;
    out_idx[q * k + r] = best >= 0 ? bi : -1;
    if (out_dist) out_dist[q * k + r] = best >= 0 ? bd : FLT_MAX;
  }
}

__global__ void init_centroids_kernel(const float *__restrict__ X, int64_t M, int N, int nlist, float *__restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nlist * N) return;
  const int64_t c = e / N;
  const int d = (int)(e % N);
  C[e] = X[(c * M / nlist) * N + d];
}

// centroid c <- mean of the points of list c, summed in list order (ids
// ascending); an empty list keeps its centroid
__global__ void centroid_mean_kernel(const float *__restrict__ X, int N, const int32_t *__restrict__ lptr,
                                     const int32_t *__restrict__ pos_id, float *__restrict__ C) {
  const int c = blockIdx.x;
  const int32_t b = lptr[c], e = lptr[c + 1];
  if (e == b) return;
  const float inv = 1.f / (float)(e - b);
  for (int d = threadIdx.x; d < N; d += blockDim.x) {
    float s = 0.f;
    for (int32_t p = b; p < e; ++p) s += X[(int64_t)pos_id[p] * N + d];
    C[(int64_t)c * N + d] = s * inv;
  }
}

template <int KP>
hipError_t launch_knn_kp(const float *X, int64_t M, int N, const float *Q, int64_t nq, const _Float16 *Xh,
                         const _Float16 *Xl, const _Float16 *Qh, const _Float16 *Ql, int Np, float inv_scale2,
                         int self_mode, const int32_t *self, const float *cnorm, int k, int32_t *idx, float *dist,
                         hipStream_t s) {
  static_assert(2 * QB * KP <= QB * SP, "merge buffers must fit in the score tile");
  const unsigned grid = (unsigned)((nq + QB - 1) / QB);
#define IVHD_SMALL_ARGS X, M, N, Q, nq, Xh, Xl, Qh, Ql, inv_scale2, self_mode, self, cnorm, k, idx, dist
  // (KP = 32 with four K steps would spill registers: the general kernel)
  if (Np == TKK) {
    knn_small_kernel<KP, 1><<<grid, kKnnThreads, 0, s>>>(IVHD_SMALL_ARGS);
  } else if (Np == 2 * TKK) {
    knn_small_kernel<KP, 2><<<grid, kKnnThreads, 0, s>>>(IVHD_SMALL_ARGS);
  } else if (Np == 3 * TKK) {
    knn_small_kernel<KP, 3><<<grid, kKnnThreads, 0, s>>>(IVHD_SMALL_ARGS);
  } else if constexpr (KP < 32) {
    if (Np == 4 * TKK) knn_small_kernel<KP, 4><<<grid, kKnnThreads, 0, s>>>(IVHD_SMALL_ARGS);
    else knn_kernel<KP><<<grid, kKnnThreads, 0, s>>>(X, M, N, Q, nq, Xh, Xl, Qh, Ql, Np, inv_scale2, self_mode,
                                                      self, cnorm, k, idx, dist);
  } else {
    knn_kernel<KP><<<grid, kKnnThreads, 0, s>>>(X, M, N, Q, nq, Xh, Xl, Qh, Ql, Np, inv_scale2, self_mode, self,
                                                 cnorm, k, idx, dist);
  }
#undef IVHD_SMALL_ARGS
  return hipGetLastError();
}

}  // namespace

int knn_max_k() { return 28; }

int knn_padded_width(int N) { return (N + TKK - 1) / TKK * TKK; }

hipError_t launch_row_norms(const float *X, int64_t M, int N, float *out, hipStream_t s) {
  row_norms_kernel<<<grid_for(M, 4), 256, 0, s>>>(X, M, N, out);
  return hipGetLastError();
}

hipError_t launch_absmax(const float *X, int64_t n, uint32_t *out, hipStream_t s) {
  absmax_kernel<<<1024, 256, 0, s>>>(X, n, out);
  return hipGetLastError();
}

// 2^s with the largest scaled magnitude below 2^kSplitMaxExp; |s| <= 60 so
// that 1 / scale^2 is a normal float (beyond that range squared distances
// overflow or vanish in FP32 anyway)
float knn_split_scale(float absmax) {
  if (!(absmax > 0.f)) return 1.f;
  int e;
  (void)frexpf(absmax, &e);   // absmax = m 2^e, 0.5 <= m < 1
  int sh = kSplitMaxExp - e;
  sh = sh > 60 ? 60 : (sh < -60 ? -60 : sh);
  return ldexpf(1.f, sh);
}

hipError_t launch_split(const float *X, int64_t M, int N, int Np, float scale, _Float16 *hi, _Float16 *lo,
                        hipStream_t s) {
  split_kernel<<<grid_for(M * Np), kBlock, 0, s>>>(X, M, N, Np, scale, hi, lo);
  return hipGetLastError();
}

hipError_t launch_knn(const float *X, int64_t M, int N, const float *Q, int64_t nq, const _Float16 *Xh,
                      const _Float16 *Xl, const _Float16 *Qh, const _Float16 *Ql, int Np, float scale,
                      int self_mode, const int32_t *self, const float *cnorm, int k, int32_t *idx, float *dist,
                      hipStream_t s) {
  const float inv2 = 1.f / (scale * scale);
  if (k + 4 <= 8)
    return launch_knn_kp<8>(X, M, N, Q, nq, Xh, Xl, Qh, Ql, Np, inv2, self_mode, self, cnorm, k, idx, dist, s);
  if (k + 4 <= 16)
    return launch_knn_kp<16>(X, M, N, Q, nq, Xh, Xl, Qh, Ql, Np, inv2, self_mode, self, cnorm, k, idx, dist, s);
  return launch_knn_kp<32>(X, M, N, Q, nq, Xh, Xl, Qh, Ql, Np, inv2, self_mode, self, cnorm, k, idx, dist, s);
}

hipError_t launch_gather_f32(const float *src, const int32_t *idx, int64_t n, float *dst, hipStream_t s) {
  gather_f32_kernel<<<grid_for(n), kBlock, 0, s>>>(src, idx, n, dst);
  return hipGetLastError();
}

hipError_t launch_split_gather(const float *X, int64_t M, int N, int Np, float scale, const int32_t *pos_id,
                               _Float16 *hi, _Float16 *lo, hipStream_t s) {
  split_gather_kernel<<<grid_for(M * Np), kBlock, 0, s>>>(X, M, N, Np, scale, pos_id, hi, lo);
  return hipGetLastError();
}

hipError_t launch_ivf_lists(const float *X, int N, const float *Q, const _Float16 *Xh, const _Float16 *Xl,
                            const _Float16 *Qh, const _Float16 *Ql, int Np, float scale, const float *pnorm,
                            const int32_t *pos_id, const int32_t *lptr, const int32_t *pptr, const int32_t *pq,
                            const int32_t *work_list, const int32_t *work_chunk, int64_t n_work,
                            const int32_t *probes, int nprobe, const int32_t *self, int k, int32_t *part_idx,
                            float *part_dist, hipStream_t s) {
  if (n_work == 0) return hipSuccess;
  const float inv2 = 1.f / (scale * scale);
  const unsigned g = (unsigned)n_work;
#define IVHD_IVF_ARGS X, N, Q, Xh, Xl, Qh, Ql, Np, inv2, pnorm, pos_id, lptr, pptr, pq, work_list, work_chunk, \
                      probes, nprobe, self, k, part_idx, part_dist
  if (k + 4 <= 8) ivf_list_kernel<8><<<g, kKnnThreads, 0, s>>>(IVHD_IVF_ARGS);
  else if (k + 4 <= 16) ivf_list_kernel<16><<<g, kKnnThreads, 0, s>>>(IVHD_IVF_ARGS);
  else ivf_list_kernel<32><<<g, kKnnThreads, 0, s>>>(IVHD_IVF_ARGS);
#undef IVHD_IVF_ARGS
  return hipGetLastError();
}

hipError_t launch_ivf_merge(const int32_t *part_idx, const float *part_dist, int64_t nq, int nprobe, int k,
                            int32_t *idx, float *dist, hipStream_t s) {
  ivf_merge_kernel<<<grid_for(nq), kBlock, 0, s>>>(part_idx, part_dist, nq, nprobe, k, idx, dist);
  return hipGetLastError();
}

hipError_t launch_init_centroids(const float *X, int64_t M, int N, int nlist, float *C, hipStream_t s) {
  init_centroids_kernel<<<grid_for((int64_t)nlist * N), kBlock, 0, s>>>(X, M, N, nlist, C);
  return hipGetLastError();
}

hipError_t launch_centroid_mean(const float *X, int N, const int32_t *lptr, const int32_t *pos_id, int nlist,
                                float *C, hipStream_t s) {
  centroid_mean_kernel<<<(unsigned)nlist, kBlock, 0, s>>>(X, N, lptr, pos_id, C);
  return hipGetLastError();
}

}  // namespace ivhd
