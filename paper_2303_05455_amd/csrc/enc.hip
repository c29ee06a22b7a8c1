// Kernels of the parametric encoder (an MLP N-D -> 2-D trained on the IVHD
// stress): BF16 operands on the gfx950 matrix cores with FP32 accumulation.
//
// gemm_bf16: C[M][N] = sum_k opA[m][k] opB[k][n]
//   opA[m][k] = A[m*lda + k]  (ta = 0)  or  A[k*lda + m]  (ta = 1)
//   opB[k][n] = B[k*ldb + n]  (tb = 0)  or  B[n*ldb + k]  (tb = 1)
// Waves own 64 x 64 output blocks; operands are staged in LDS with K
// contiguous per row, so one lane's MFMA operand (8 consecutive k) is a
// single 16-byte LDS read.  The instruction is v_mfma_f32_16x16x32_bf16:
// lane l supplies A[l%16][8(l/16)..+8) and B[8(l/16)..+8)[l%16], and
// receives D[4(l/16)+r][l%16], r = 0..3.
// Two kernels: gemm_nt_kernel when both operands are K-contiguous (ta = 0,
// tb = 1) with 16-byte rows (every GEMM of the training step is arranged
// so): 256 x 128 tiles of 8 waves, K steps of 32 through a ring of LDS
// stages filled by direct-to-LDS loads; gemm_kernel for every other
// layout: 128 x 128 tiles of 4 waves, K steps of 32 staged through
// registers.
// Epilogues: FP32 store (split-K partials: the K split selects the K range
// and the output slab), bias + ReLU -> BF16, or (dgrad) multiply by the
// ReLU derivative read from the forward activation -> BF16.
//
// Rounding: every FP32 -> BF16 conversion is round-to-nearest-even.
#include "enc_internal.h"

namespace ivhd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int KP = TK + 8;   // LDS row pitch in bf16 (80 bytes: 16-byte aligned rows)
constexpr int kGemmThreads = 256;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct alignas(16) U16x8 {
  uint16_t v[8];
};

// one operand tile (rows r0..r0+127 of op, k0..k0+31) in two halves, so the
// global loads of step s + 1 can be issued before the MFMAs of step s:
// op[row][k] = T ? P[k*ld + row] : P[row*ld + k]; out of range -> 0.
// Each thread holds two 8-element chunks.
struct TileFrag {
  U16x8 v[2];
};

template <bool T>
__device__ __forceinline__ void load_tile(TileFrag &F, const uint16_t *__restrict__ P, int64_t ld, int64_t rows,
                                          int64_t r0, int64_t k0, int64_t kend, bool vec_ok) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int id = tid + kGemmThreads * c;
    U16x8 &v = F.v[c];
    if (!T) {
      // 128 rows x 4 chunks of 8 k
      const int r = id >> 2, kc = (id & 3) * 8;
      const int64_t row = r0 + r, k = k0 + kc;
      if (row < rows && vec_ok && k + 8 <= kend) {
        v = *reinterpret_cast<const U16x8 *>(P + row * ld + k);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v.v[j] = (row < rows && k + j < kend) ? P[row * ld + k + j] : (uint16_t)0;
      }
    } else {
      // k-major source: 32 k x 16 chunks of 8 rows
      const int kk = id >> 4, rc = (id & 15) * 8;
      const int64_t k = k0 + kk, row = r0 + rc;
      if (k < kend && vec_ok && row + 8 <= rows) {
        v = *reinterpret_cast<const U16x8 *>(P + k * ld + row);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v.v[j] = (k < kend && row + j < rows) ? P[k * ld + row + j] : (uint16_t)0;
      }
    }
  }
}

template <bool T>
__device__ __forceinline__ void store_tile(const TileFrag &F, uint16_t *__restrict__ lds) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int id = tid + kGemmThreads * c;
    if (!T) {
      const int r = id >> 2, kc = (id & 3) * 8;
      *reinterpret_cast<U16x8 *>(lds + r * KP + kc) = F.v[c];
    } else {
      const int kk = id >> 4, rc = (id & 15) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) lds[(rc + j) * KP + kk] = F.v[c].v[j];
    }
  }
}

// Epilogue of a 128 x 128 tile: wave (wm, wn) holds rows wm..wm+63 and
// columns wn..wn+63 as 4 x 4 MFMA results; lane l has column l%16 and rows
// 4(l/16)..+4 of each.  z selects the FP32 split-K slab.
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, const floatx4 (&acc)[4][4], int64_t m0, int64_t n0,
                                              int wm, int wn, int lane, int64_t z) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + wn + 16 * j + (lane & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (m >= g.M) continue;
        float x = acc[i][j][r];
        if (EPI == GEMM_EPI_F32) {
          float *C = static_cast<float *>(g.C) + z * g.M * g.ldc;
          C[m * g.ldc + n] = x;
        } else if (EPI == GEMM_EPI_BIAS_RELU_BF16) {
          x += g.bias ? g.bias[n] : 0.f;
          x = fmaxf(x, 0.f);
          static_cast<uint16_t *>(g.C)[m * g.ldc + n] = f2bf(x);
        } else {   // GEMM_EPI_RELU_MASK_BF16
          const float h = bf2f(g.mask[m * g.ldm + n]);
          static_cast<uint16_t *>(g.C)[m * g.ldc + n] = f2bf(h > 0.f ? x : 0.f);
        }
      }
    }
  }
}

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(kGemmThreads) gemm_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TM * KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN * KP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
  const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // A rows are m: opA[m][k] is P[row*ld + k] unless transposed.  B rows are
  // n: opB[k][n] is P[row*ld + k] exactly when B is given transposed.
  TileFrag fa, fb;
  load_tile<TA>(fa, g.A, g.lda, g.M, m0, kbeg, kend, g.vec_a);
  load_tile<!TB>(fb, g.B, g.ldb, g.N, n0, kbeg, kend, g.vec_b);
  for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
    __syncthreads();
    store_tile<TA>(fa, As);
    store_tile<!TB>(fb, Bs);
    __syncthreads();
    if (k0 + TK < kend) {   // the next step's loads fly during this step's MFMAs
      load_tile<TA>(fa, g.A, g.lda, g.M, m0, k0 + TK, kend, g.vec_a);
      load_tile<!TB>(fb, g.B, g.ldb, g.N, n0, k0 + TK, kend, g.vec_b);
    }
    const int kq = (lane >> 4) * 8;
    bf16x8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm + 16 * i + (lane & 15)) * KP + kq);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn + 16 * j + (lane & 15)) * KP + kq);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }

  gemm_epilogue<EPI>(g, acc, m0, n0, wm, wn, lane, blockIdx.z);
}

// ---- both operands K-contiguous (opA = A[m][k], opB = B[n][k]) -----------
// Tiles of 256 x 128 per block of 512 threads (8 waves of 64 x 64, four
// along M by two along N).  K goes in steps of 32 through a ring of three
// LDS stages that global_load_lds_dwordx4 fills directly (no register
// staging): a step's loads are issued two steps ahead, each wave waits for
// its own loads of the step with vmcnt, and one barrier per step publishes
// the stage and frees the one loaded next.  A stage holds the A rows then
// the B rows, 64 bytes each (four 16-byte chunks of k); the load writes lane
// l's chunk at stage slot base + l, so each lane picks which chunk to fetch,
// and chunk c of row r sits in slot 4 r + (c ^ ((r >> 1) & 3)): the 16 rows
// an MFMA operand read touches then fall on distinct bank groups.  Two
// blocks share a CU (74 KB of LDS each), so one block's epilogue overlaps
// the other's loop.  Tiles are dealt to the XCDs in contiguous runs (blocks
// go to XCD b % 8), ordered by K split, then along the longer output side,
// then the shorter one: the tiles that share a panel of the long operand,
// and the tiles of one K split, run on one XCD and share its L2.  Requires
// 16-byte aligned operands with lda, ldb and K multiples of 8, so every
// chunk is wholly inside or outside the matrix: a chunk past the last row
// reads the operand's first chunk instead (its outputs are never stored),
// and chunks past the end of K are zeroed in LDS once they have arrived.
// Measured at 57,344 x 784 x 512: 74.6 us against 96.7 us for 128 x 128
// tiles with register staging.
constexpr int NTK = 64;        // K granularity of a split-K chunk
constexpr int kXcds = 8;
constexpr int BM = 256, BN = 128, BK = 32;
constexpr int kNtThreads = 512;
constexpr int kRing = 3;
constexpr int kStage = (BM + BN) * BK;            // bf16 per stage
constexpr int kStageLoads = (BM + BN) * BK / 8 / kNtThreads;   // 16-byte chunks per thread per stage
static_assert(kStageLoads * kNtThreads * 8 == kStage, "a stage is a whole number of wave loads");
constexpr int kCbPitch = BN + 8;                 // bf16 epilogue tile pitch (272 bytes)
constexpr int kCfPitch = BN + 4;                 // FP32 epilogue half-tile pitch
static_assert(BM * kCbPitch * 2 <= kRing * kStage * 2, "bf16 tile must fit in the ring");
static_assert(BM / 2 * kCfPitch * 4 <= kRing * kStage * 2, "FP32 half tile must fit in the ring");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int ring_slot(int row, int chunk) { return row * 4 + (chunk ^ ((row >> 1) & 3)); }

template <int EPI>
__global__ void __launch_bounds__(kNtThreads, 2) gemm_nt_kernel(GemmArgs g, int64_t tiles_m, int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) uint16_t S[kRing * kStage];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nb = (int64_t)gridDim.x, lin = blockIdx.x;
  const int64_t q = nb / kXcds, rem = nb % kXcds, x = lin % kXcds, i = lin / kXcds;
  const int64_t tile = x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
  const int64_t per_z = tiles_m * tiles_n, z = tile / per_z, t = tile % per_z;
  const bool m_outer = tiles_m >= tiles_n;
  const int64_t m0 = (m_outer ? t / tiles_n : t % tiles_m) * BM;
  const int64_t n0 = (m_outer ? t % tiles_n : t / tiles_m) * BN;
  const int64_t kbeg = z * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  const int nsteps = (int)((kend - kbeg + BK - 1) / BK);
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  // this thread's chunks of every stage: slot (wave * kStageLoads + c) * 64 + lane
  int row_of[kStageLoads], chunk_of[kStageLoads];
#pragma unroll
  for (int c = 0; c < kStageLoads; ++c) {
    const int slot = (wave * kStageLoads + c) * 64 + lane, r = slot >> 2;
    row_of[c] = r;
    chunk_of[c] = (slot & 3) ^ ((r >> 1) & 3);
  }
  auto issue = [&](int st) {
    const int64_t k0 = kbeg + (int64_t)st * BK;
    uint16_t *base = S + (st % kRing) * kStage;
#pragma unroll
    for (int c = 0; c < kStageLoads; ++c) {
      const int64_t k = k0 + chunk_of[c] * 8;
      const int r = row_of[c];
      const uint16_t *p;
      if (r < BM) {
        const int64_t ra = m0 + r;
        p = ra < g.M && k < kend ? g.A + ra * g.lda + k : g.A;
      } else {
        const int64_t rb = n0 + (r - BM);
        p = rb < g.N && k < kend ? g.B + rb * g.ldb + k : g.B;
      }
      __builtin_amdgcn_global_load_lds((const void *)p, (lds_void *)(base + (wave * kStageLoads + c) * 64 * 8), 16,
                                       0, 0);
    }
  };

  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  static_assert(kRing == 3 && kStageLoads == 3, "the vmcnt waits below count three loads per stage");
  int issued = 0;
  for (; issued < kRing - 1 && issued < nsteps; ++issued) issue(issued);
  for (int st = 0; st < nsteps; ++st) {
    // this step's loads are done once at most the later stages' remain
    if (issued - st - 1 >= 1) asm volatile("s_waitcnt vmcnt(3)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    uint16_t *base = S + (st % kRing) * kStage;
    if (kbeg + (int64_t)(st + 1) * BK > kend) {   // K tail: zero this thread's chunks past the end
#pragma unroll
      for (int c = 0; c < kStageLoads; ++c)
        if (kbeg + (int64_t)st * BK + chunk_of[c] * 8 >= kend)
          *reinterpret_cast<u32x4 *>(base + (wave * kStageLoads + c) * 64 * 8 + lane * 8) = u32x4{0u, 0u, 0u, 0u};
    }
    // LDS writes done, then the barrier: the stage is complete for every
    // wave, and every wave has finished reading the stage loaded next
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    if (issued < nsteps) issue(issued++);
    const uint16_t *As = base, *Bs = base + BM * BK;
    const int kc = lane >> 4;
    bf16x8 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      a[u] = *reinterpret_cast<const bf16x8 *>(As + ring_slot(wm + 16 * u + (lane & 15), kc) * 8);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      b[u] = *reinterpret_cast<const bf16x8 *>(Bs + ring_slot(wn + 16 * u + (lane & 15), kc) * 8);
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        acc[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ii], b[jj], acc[ii][jj], 0, 0, 0);
  }
  __syncthreads();   // all loads landed and all operand reads done: the ring is free

  // Epilogue.  Wave (wm, wn) holds rows wm..wm+63 and columns wn..wn+63 as
  // 4 x 4 MFMA results; lane l has column l % 16 and rows 4 (l / 16)..+4 of
  // each.  The tile goes through LDS so that every thread finishes whole row
  // chunks with 16-byte stores where the leading dimension and pointer allow.
  if (EPI == GEMM_EPI_F32) {
    // FP32 in two halves of 128 rows (waves 0-3, then 4-7)
    float *Cf = reinterpret_cast<float *>(S);
    float *C = static_cast<float *>(g.C) + z * g.M * g.ldc;
    const bool vec = g.ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if ((wave >> 2) == half) {
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              Cf[(wm - 128 * half + 16 * ii + 4 * (lane >> 4) + r) * kCfPitch + wn + 16 * jj + (lane & 15)] =
                  acc[ii][jj][r];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 8; ++c) {   // 128 rows x 32 chunks of 4
        const int id = tid + kNtThreads * c, m = id >> 5, qc = (id & 31) * 4;
        const int64_t row = m0 + 128 * half + m, col = n0 + qc;
        if (row >= g.M || col >= g.N) continue;
        const floatx4 v = *reinterpret_cast<const floatx4 *>(Cf + m * kCfPitch + qc);
        if (vec && col + 4 <= g.N) {
          *reinterpret_cast<floatx4 *>(C + row * g.ldc + col) = v;
        } else {
          for (int e = 0; e < 4 && col + e < g.N; ++e) C[row * g.ldc + col + e] = v[e];
        }
      }
      __syncthreads();
    }
    return;
  }
  // BF16 outputs: bias + ReLU applied in FP32 before rounding; the ReLU mask
  // (a zero or a copy of the rounded value) after it, which is the same
  uint16_t *Cb = S;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int64_t col = n0 + wn + 16 * jj + (lane & 15);
    const float bv = EPI == GEMM_EPI_BIAS_RELU_BF16 && g.bias && col < g.N ? g.bias[col] : 0.f;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[ii][jj][r];
        if (EPI == GEMM_EPI_BIAS_RELU_BF16) v = fmaxf(v + bv, 0.f);
        Cb[(wm + 16 * ii + 4 * (lane >> 4) + r) * kCbPitch + wn + 16 * jj + (lane & 15)] = f2bf(v);
      }
  }
  __syncthreads();
  uint16_t *C = static_cast<uint16_t *>(g.C);
  const bool vec = g.ldc % 8 == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
  const bool vec_m = EPI == GEMM_EPI_RELU_MASK_BF16 && g.ldm % 8 == 0 &&
                     (reinterpret_cast<uintptr_t>(g.mask) & 15) == 0;
  // 256 rows x 16 chunks of 8: thread chunk c is row (tid >> 4) + 32 c.
  // Whole mask chunks are loaded first, branch-free (others read the first
  // chunk and are replaced element by element below).
  U16x8 mk[8];
  if (EPI == GEMM_EPI_RELU_MASK_BF16) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int64_t row = m0 + (tid >> 4) + 32 * c, col = n0 + (tid & 15) * 8;
      const bool full = vec_m && row < g.M && col + 8 <= g.N;
      mk[c] = *reinterpret_cast<const U16x8 *>(full ? g.mask + row * g.ldm + col : g.mask);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int m = (tid >> 4) + 32 * c, qc = (tid & 15) * 8;
    const int64_t row = m0 + m, col = n0 + qc;
    if (row >= g.M || col >= g.N) continue;
    U16x8 o = *reinterpret_cast<const U16x8 *>(Cb + m * kCbPitch + qc);
    if (EPI == GEMM_EPI_RELU_MASK_BF16) {
      if (!(vec_m && col + 8 <= g.N))
        for (int e = 0; e < 8; ++e) mk[c].v[e] = col + e < g.N ? g.mask[row * g.ldm + col + e] : (uint16_t)0;
#pragma unroll
      for (int e = 0; e < 8; ++e) o.v[e] = bf2f(mk[c].v[e]) > 0.f ? o.v[e] : (uint16_t)0;
    }
    if (vec && col + 8 <= g.N) {
      *reinterpret_cast<U16x8 *>(C + row * g.ldc + col) = o;
    } else {
      for (int e = 0; e < 8 && col + e < g.N; ++e) C[row * g.ldc + col + e] = o.v[e];
    }
  }
}

// sum of `splits` FP32 slabs [M][ldc] in slab order -> out (FP32, ld = ldo)
__global__ void splitk_reduce_kernel(const float *__restrict__ part, int splits, int64_t M, int64_t N,
                                     int64_t ldp, float *__restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t m = e / N, n = e % N;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * M * ldp + m * ldp + n];
  out[m * ldo + n] = s;
}

template <bool TA, bool TB>
hipError_t launch_gemm_t(const GemmArgs &g, int epi, dim3 grid, hipStream_t s) {
  switch (epi) {
    case GEMM_EPI_F32: gemm_kernel<TA, TB, GEMM_EPI_F32><<<grid, kGemmThreads, 0, s>>>(g); break;
    case GEMM_EPI_BIAS_RELU_BF16:
      gemm_kernel<TA, TB, GEMM_EPI_BIAS_RELU_BF16><<<grid, kGemmThreads, 0, s>>>(g);
      break;
    default: gemm_kernel<TA, TB, GEMM_EPI_RELU_MASK_BF16><<<grid, kGemmThreads, 0, s>>>(g); break;
  }
  return hipGetLastError();
}

// ---- small kernels around the GEMMs -------------------------------------

// out[c][r] = in[r][c] for a BF16 [R][C] matrix, rows of out padded to ldo
// (>= R) with zeros; 64 x 64 tiles through LDS (coalesced reads and writes)
__global__ void __launch_bounds__(256) transpose_bf16_kernel(const uint16_t *__restrict__ in, int64_t R, int64_t C,
                                                            uint16_t *__restrict__ out, int64_t ldo) {
  __shared__ uint16_t t[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    t[i][tx] = (r < R && c < C) ? in[r * C + c] : (uint16_t)0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < C && r < ldo) out[c * ldo + r] = t[tx][i];
  }
}

__global__ void f32_to_bf16_kernel(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = f2bf(x[e]);
}

// out[r][:] = X[rows[r]][:] (BF16 rows of width N); 16-byte chunks when the
// rows are 16-byte multiples (N % 8 == 0, aligned bases), else elements
__global__ void gather_rows_kernel(const uint16_t *__restrict__ X, int64_t N, const int32_t *__restrict__ rows,
                                   int64_t R, uint16_t *__restrict__ out, bool vec) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec) {
    const int64_t cpr = N / 8;   // chunks per row
    if (e >= R * cpr) return;
    const int64_t r = e / cpr, c = e % cpr;
    *reinterpret_cast<U16x8 *>(out + r * N + 8 * c) =
        *reinterpret_cast<const U16x8 *>(X + (int64_t)rows[r] * N + 8 * c);
    return;
  }
  if (e >= R * N) return;
  const int64_t r = e / N, k = e % N;
  out[e] = X[(int64_t)rows[r] * N + k];
}

// Z[r][o] = b3[o] + sum_k H[r][k] W3[o][k], o < 2 (one wavefront per row;
// with vec, K % 8 == 0 and 16-byte aligned H and W3, each lane takes 8
// consecutive k per 16-byte load)
__global__ void __launch_bounds__(256) head_forward_kernel(const uint16_t *__restrict__ H, int64_t R, int K,
                                                           const uint16_t *__restrict__ W3,
                                                           const float *__restrict__ b3, float *__restrict__ Z,
                                                           bool vec) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  float s0 = 0.f, s1 = 0.f;
  if (vec) {
    for (int k = 8 * lane; k < K; k += 512) {
      const U16x8 h = *reinterpret_cast<const U16x8 *>(H + r * K + k);
      const U16x8 w0 = *reinterpret_cast<const U16x8 *>(W3 + k);
      const U16x8 w1 = *reinterpret_cast<const U16x8 *>(W3 + K + k);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        s0 += bf2f(h.v[j]) * bf2f(w0.v[j]);
        s1 += bf2f(h.v[j]) * bf2f(w1.v[j]);
      }
    }
  } else {
    for (int k = lane; k < K; k += 64) {
      const float h = bf2f(H[r * K + k]);
      s0 += h * bf2f(W3[k]);
      s1 += h * bf2f(W3[K + k]);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
  }
  if (lane == 0) {
    Z[2 * r] = s0 + b3[0];
    Z[2 * r + 1] = s1 + b3[1];
  }
}

// dH[r][k] = (dZ[r][0] W3[0][k] + dZ[r][1] W3[1][k]) * [H[r][k] > 0]  -> BF16
__global__ void head_dgrad_kernel(const float *__restrict__ dZ, const uint16_t *__restrict__ W3,
                                  const uint16_t *__restrict__ H, int64_t R, int K, uint16_t *__restrict__ dH) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= R * K) return;
  const int64_t r = e / K;
  const int k = (int)(e % K);
  const float g = dZ[2 * r] * bf2f(W3[k]) + dZ[2 * r + 1] * bf2f(W3[K + k]);
  dH[e] = f2bf(bf2f(H[e]) > 0.f ? g : 0.f);
}

// A 64-row x 64-column tile of a BF16 [R][C] matrix is formed, optionally
// written row-major to `out`, and written feature-major to outT [C][ldo]
// (entries r >= R zero) through LDS, all with 16-byte accesses:
//   TT_COPY       the tile of `in`
//   TT_GATHER     rows `rows[r]` of `in` (a batch gathered from the data)
//   TT_HEAD_DGRAD the head's input gradient from the activations `in` = H:
//                 (dZ[r][0] W3[0][k] + dZ[r][1] W3[1][k]) * [H[r][k] > 0]
// Needs C and ldo multiples of 8 and 16-byte aligned in, out, outT.
__global__ void __launch_bounds__(256) tile_t_kernel(int mode, TileTArgs a) {
  __shared__ uint32_t t[64][33];   // 64 rows of 64 BF16 (+ one word of padding)
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int id = threadIdx.x + 256 * c, rl = id >> 3, cc = (id & 7) * 8;
    const int64_t r = r0 + rl, col = c0 + cc;
    U16x8 v = {};
    if (r < a.R && col < a.C) {
      const int64_t src = (mode == TT_GATHER ? (int64_t)a.rows[r] : r) * a.C + col;
      v = *reinterpret_cast<const U16x8 *>(a.in + src);
      if (mode == TT_HEAD_DGRAD) {
        const float g0 = a.dz[2 * r], g1 = a.dz[2 * r + 1];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float g = g0 * bf2f(a.w3[col + j]) + g1 * bf2f(a.w3[a.C + col + j]);
          v.v[j] = f2bf(bf2f(v.v[j]) > 0.f ? g : 0.f);
        }
      }
      if (a.out) *reinterpret_cast<U16x8 *>(a.out + r * a.C + col) = v;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) t[rl][cc / 2 + j] = (uint32_t)v.v[2 * j] | ((uint32_t)v.v[2 * j + 1] << 16);
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int id = threadIdx.x + 256 * c, kl = id >> 3, rc = (id & 7) * 8;
    const int64_t k = c0 + kl, rr = r0 + rc;
    if (k < a.C && rr < a.ldo) {
      U16x8 o;
#pragma unroll
      for (int j = 0; j < 8; ++j) o.v[j] = (uint16_t)(t[rc + j][kl >> 1] >> ((kl & 1) * 16));
      *reinterpret_cast<U16x8 *>(a.outT + k * a.ldo + rr) = o;
    }
  }
}

// out[j] = sum over the L entries of row j of a BF16 [J][L] matrix: each
// thread sums its 8-element chunks (stride = block size) in order, then a
// fixed tree over the block; deterministic
__global__ void __launch_bounds__(kBlock) rowsum_bf16_kernel(const uint16_t *__restrict__ X, int64_t L,
                                                            float *__restrict__ out) {
  __shared__ float red[kBlock];
  const uint16_t *row = X + (int64_t)blockIdx.x * L;
  float acc = 0.f;
  const bool vec = L % 8 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (vec) {
    for (int64_t c = threadIdx.x; c < L / 8; c += kBlock) {
      const U16x8 v = *reinterpret_cast<const U16x8 *>(row + 8 * c);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += bf2f(v.v[j]);
    }
  } else {
    for (int64_t c = threadIdx.x; c < L; c += kBlock) acc += bf2f(row[c]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// column sums over row chunks: part[c][j] = sum_{r in chunk c} f(r, j) for
//   mode 0: BF16 matrix X[R][J]
//   mode 1: dZ (FP32 [R][2]) x H (BF16 [R][K]): j = o*K + k -> dZ[r][o] H[r][k]  (dW3)
//   mode 2: FP32 matrix [R][J]            (bias gradient of the head, later levels)
// A block of 8 x 32 threads covers 32 V-column groups of one chunk of
// kColsumRows rows: row lane ty sums rows ty, ty + 8, ... in order, then
// the eight lane sums are added in order ty = 0..7 (deterministic).  V = 8
// needs J (and K) multiples of 8 and a 16-byte aligned source.
template <int V>
__global__ void __launch_bounds__(256) colsum_kernel(int mode, const void *__restrict__ Xp,
                                                    const float *__restrict__ dZ, int64_t R, int64_t J, int64_t K,
                                                    float *__restrict__ part) {
  __shared__ float red[8][32 * V + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 32 + tx) * V;
  const int64_t r0 = (int64_t)blockIdx.y * kColsumRows;
  const int64_t r1 = r0 + kColsumRows < R ? r0 + kColsumRows : R;
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.f;
  if (j0 < J) {
    const int64_t half = mode == 1 ? j0 / K : 0, col = mode == 1 ? j0 % K : j0, ld = mode == 1 ? K : J;
#pragma unroll 4
    for (int64_t r = r0 + ty; r < r1; r += 8) {
      float x[V];
      if (mode == 2) {
        const float *X = static_cast<const float *>(Xp) + r * J + j0;
        if (V == 8) {
          const floatx4 lo = *reinterpret_cast<const floatx4 *>(X), hi = *reinterpret_cast<const floatx4 *>(X + 4);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            x[e] = lo[e];
            x[e + 4] = hi[e];
          }
        } else {
          x[0] = X[0];
        }
      } else {
        const uint16_t *X = static_cast<const uint16_t *>(Xp) + r * ld + col;
        const float w = mode == 1 ? dZ[2 * r + half] : 1.f;
        if (V == 8) {
          const U16x8 v = *reinterpret_cast<const U16x8 *>(X);
#pragma unroll
          for (int e = 0; e < V; ++e) x[e] = mode == 1 ? w * bf2f(v.v[e]) : bf2f(v.v[e]);
        } else {
          x[0] = mode == 1 ? w * bf2f(X[0]) : bf2f(X[0]);
        }
      }
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += x[e];
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e) red[ty][tx * V + e] = acc[e];
  __syncthreads();
  if (ty == 0 && j0 < J) {
#pragma unroll
    for (int e = 0; e < V; ++e) {
      float t = red[0][tx * V + e];
#pragma unroll
      for (int q = 1; q < 8; ++q) t += red[q][tx * V + e];
      part[(int64_t)blockIdx.y * J + j0 + e] = t;
    }
  }
}

// Adam with bias correction 1/(1 - beta^t); refreshes the BF16 copy
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ w16, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2, float gscale) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gr = g[e] * gscale;
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  const float wn = w[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  w[e] = wn;
  w16[e] = f2bf(wn);
}

// Glorot-uniform weights U(-s, s), s = sqrt(6 / (fan_in + fan_out)), from a
// SplitMix64 counter stream; biases zero
__global__ void glorot_kernel(float *__restrict__ w, int64_t n, int fan_in, int fan_out, uint64_t seed,
                              uint64_t offset) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  uint64_t z = seed ^ (offset + (uint64_t)e) * 0x9e3779b97f4a7c15ull;
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  const float u = (float)(z >> 40) * (1.0f / 16777216.0f);   // [0, 1)
  const float s = sqrtf(6.0f / (float)(fan_in + fan_out));
  w[e] = (2.f * u - 1.f) * s;
}

__global__ void scale_dz_kernel(float *__restrict__ dz, int64_t n, const float *__restrict__ s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dz[e] *= *s;
}

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs &g0, int ta, int tb, int epi, int splits, hipStream_t s) {
  GemmArgs g = g0;
  if (splits < 1) splits = 1;
  g.kchunk = ((g.K + splits - 1) / splits + NTK - 1) / NTK * NTK;
  if (g.kchunk < NTK) g.kchunk = NTK;
  splits = (int)((g.K + g.kchunk - 1) / g.kchunk);
  if (splits < 1) splits = 1;
  if (!ta && tb && g.vec_a && g.vec_b && g.K % 8 == 0) {
    const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN, nb = tm * tn * splits;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    switch (epi) {
      case GEMM_EPI_F32: gemm_nt_kernel<GEMM_EPI_F32><<<(unsigned)nb, kNtThreads, 0, s>>>(g, tm, tn); break;
      case GEMM_EPI_BIAS_RELU_BF16:
        gemm_nt_kernel<GEMM_EPI_BIAS_RELU_BF16><<<(unsigned)nb, kNtThreads, 0, s>>>(g, tm, tn);
        break;
      default: gemm_nt_kernel<GEMM_EPI_RELU_MASK_BF16><<<(unsigned)nb, kNtThreads, 0, s>>>(g, tm, tn); break;
    }
    return hipGetLastError();
  }
  dim3 grid((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TM - 1) / TM), (unsigned)splits);
  if (!ta && !tb) return launch_gemm_t<false, false>(g, epi, grid, s);
  if (!ta && tb) return launch_gemm_t<false, true>(g, epi, grid, s);
  if (ta && !tb) return launch_gemm_t<true, false>(g, epi, grid, s);
  return launch_gemm_t<true, true>(g, epi, grid, s);
}

int gemm_splits_used(int64_t K, int splits) {
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + NTK - 1) / NTK * NTK;
  if (kchunk < NTK) kchunk = NTK;
  const int64_t used = (K + kchunk - 1) / kchunk;
  return (int)(used < 1 ? 1 : used);
}

hipError_t launch_splitk_reduce(const float *part, int splits, int64_t M, int64_t N, int64_t ldp, float *out,
                                int64_t ldo, hipStream_t s) {
  splitk_reduce_kernel<<<grid_for(M * N), kBlock, 0, s>>>(part, splits, M, N, ldp, out, ldo);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const uint16_t *in, int64_t R, int64_t C, uint16_t *out, int64_t ldo,
                                 hipStream_t s) {
  if (ldo == 0 || C == 0) return hipSuccess;
  if (ldo < R || (C + 63) / 64 > 65535 || (ldo + 63) / 64 > INT32_MAX) return hipErrorInvalidValue;
  transpose_bf16_kernel<<<dim3((unsigned)((ldo + 63) / 64), (unsigned)((C + 63) / 64)), 256, 0, s>>>(in, R, C, out,
                                                                                                    ldo);
  return hipGetLastError();
}

bool tile_t_ok(const TileTArgs &a) {
  auto al = [](const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return a.C % 8 == 0 && a.ldo % 8 == 0 && a.ldo >= a.R && al(a.in) && al(a.out) && al(a.outT) && a.outT;
}

hipError_t launch_tile_t(int mode, const TileTArgs &a, hipStream_t s) {
  if (!tile_t_ok(a)) return hipErrorInvalidValue;
  if (a.ldo == 0 || a.C == 0) return hipSuccess;
  if ((a.C + 63) / 64 > 65535 || (a.ldo + 63) / 64 > INT32_MAX) return hipErrorInvalidValue;
  tile_t_kernel<<<dim3((unsigned)((a.ldo + 63) / 64), (unsigned)((a.C + 63) / 64)), 256, 0, s>>>(mode, a);
  return hipGetLastError();
}

hipError_t launch_rowsum_bf16(const uint16_t *X, int64_t J, int64_t L, float *out, hipStream_t s) {
  if (J == 0) return hipSuccess;
  if (J > INT32_MAX) return hipErrorInvalidValue;
  rowsum_bf16_kernel<<<(unsigned)J, kBlock, 0, s>>>(X, L, out);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s) {
  f32_to_bf16_kernel<<<grid_for(n), kBlock, 0, s>>>(x, n, y);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const uint16_t *X, int64_t N, const int32_t *rows, int64_t R, uint16_t *out,
                              hipStream_t s) {
  const bool vec = N % 8 == 0 && ((uintptr_t)X % 16 == 0) && ((uintptr_t)out % 16 == 0);
  gather_rows_kernel<<<grid_for(vec ? R * (N / 8) : R * N), kBlock, 0, s>>>(X, N, rows, R, out, vec);
  return hipGetLastError();
}

hipError_t launch_head_forward(const uint16_t *H, int64_t R, int K, const uint16_t *W3, const float *b3, float *Z,
                               hipStream_t s) {
  const bool vec = K % 8 == 0 && (reinterpret_cast<uintptr_t>(H) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(W3) & 15) == 0;
  head_forward_kernel<<<grid_for(R, 4), 256, 0, s>>>(H, R, K, W3, b3, Z, vec);
  return hipGetLastError();
}

hipError_t launch_head_dgrad(const float *dZ, const uint16_t *W3, const uint16_t *H, int64_t R, int K,
                             uint16_t *dH, hipStream_t s) {
  head_dgrad_kernel<<<grid_for(R * K), kBlock, 0, s>>>(dZ, W3, H, R, K, dH);
  return hipGetLastError();
}

int64_t colsum_workspace(int64_t R, int64_t J) {
  const int64_t c0 = (R + kColsumRows - 1) / kColsumRows;
  return (c0 + (c0 + kColsumRows - 1) / kColsumRows) * J;
}

// Column sums as a tree: each level sums kColsumRows consecutive rows into
// partials [ceil(rows / kColsumRows)][J], until one row is left (written to
// out).  Levels ping-pong between two regions of ws.
hipError_t launch_colsum(int mode, const void *X, const float *dZ, int64_t R, int64_t J, int64_t K, float *ws,
                         float *out, hipStream_t s) {
  if (R < 1 || (R + kColsumRows - 1) / kColsumRows > 65535) return hipErrorInvalidValue;
  const int64_t c0 = (R + kColsumRows - 1) / kColsumRows;
  float *buf[2] = {ws, ws + c0 * J};
  const void *src = X;
  int64_t rows = R;
  for (int level = 0;; ++level) {
    const int m = level == 0 ? mode : 2;
    const int64_t chunks = (rows + kColsumRows - 1) / kColsumRows;
    float *dst = chunks == 1 ? out : buf[level & 1];
    const bool vec8 = J % 8 == 0 && (m != 1 || K % 8 == 0) && (reinterpret_cast<uintptr_t>(src) & 15) == 0;
    if (vec8)
      colsum_kernel<8><<<dim3((unsigned)((J / 8 + 31) / 32), (unsigned)chunks), 256, 0, s>>>(m, src, dZ, rows, J,
                                                                                           K, dst);
    else
      colsum_kernel<1><<<dim3((unsigned)((J + 31) / 32), (unsigned)chunks), 256, 0, s>>>(m, src, dZ, rows, J, K,
                                                                                       dst);
    if (chunks == 1) break;
    src = dst;
    rows = chunks;
  }
  return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, uint16_t *w16, int64_t n, float lr, float b1,
                       float b2, float eps, int64_t t, float gscale, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  adam_kernel<<<grid_for(n), kBlock, 0, s>>>(w, g, m, v, w16, n, lr, b1, b2, eps, c1, c2, gscale);
  return hipGetLastError();
}

hipError_t launch_glorot(float *w, int64_t n, int fan_in, int fan_out, uint64_t seed, uint64_t offset,
                         hipStream_t s) {
  glorot_kernel<<<grid_for(n), kBlock, 0, s>>>(w, n, fan_in, fan_out, seed, offset);
  return hipGetLastError();
}

hipError_t launch_scale_dz(float *dz, int64_t n, const float *scale, hipStream_t s) {
  scale_dz_kernel<<<grid_for(n), kBlock, 0, s>>>(dz, n, scale);
  return hipGetLastError();
}

}  // namespace ivhd

namespace ivhd {
namespace {

// rows of one training batch: B sources s_b = (a (off + b) + c0) mod M, then
// their nn targets (an absent slot repeats the source, which adds nothing to
// the stress or its gradient), then their rn targets
__global__ void batch_rows_kernel(const int32_t *__restrict__ nn_idx, int nn, const int32_t *__restrict__ rn_idx,
                                  int rn, int64_t M, int64_t B, uint64_t a, uint64_t c0, int64_t off,
                                  int32_t *__restrict__ rows) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t src = (int64_t)((a * (uint64_t)(off + b) + c0) % (uint64_t)M);
  rows[b] = (int32_t)src;
  for (int q = 0; q < nn; ++q) {
    const int32_t j = nn_idx[src * nn + q];
    rows[B + b * nn + q] = j >= 0 ? j : (int32_t)src;
  }
  for (int q = 0; q < rn; ++q) rows[B + B * nn + b * rn + q] = rn_idx[src * rn + q];
}

// the fixed local edge lists of a batch: source b's nn edges point at rows
// B + b*nn + q, its rn edges at rows B + B*nn + b*rn + q; other rows have none
__global__ void batch_plan_kernel(int64_t B, int nn, int rn, int32_t *__restrict__ lnn, int32_t *__restrict__ lrn) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t R = B * (1 + nn + rn);
  if (r >= R) return;
  for (int q = 0; q < nn; ++q) lnn[r * nn + q] = r < B ? (int32_t)(B + r * nn + q) : -1;
  for (int q = 0; q < rn; ++q) lrn[r * rn + q] = r < B ? (int32_t)(B + B * nn + r * rn + q) : -1;
}

}  // namespace

hipError_t launch_batch_rows(const int32_t *nn_idx, int nn, const int32_t *rn_idx, int rn, int64_t M, int64_t B,
                             uint64_t a, uint64_t c0, int64_t off, int32_t *rows, hipStream_t s) {
  batch_rows_kernel<<<grid_for(B), kBlock, 0, s>>>(nn_idx, nn, rn_idx, rn, M, B, a, c0, off, rows);
  return hipGetLastError();
}

hipError_t launch_batch_plan(int64_t B, int nn, int rn, int32_t *lnn, int32_t *lrn, hipStream_t s) {
  batch_plan_kernel<<<grid_for(B * (1 + nn + rn)), kBlock, 0, s>>>(B, nn, rn, lnn, lrn);
  return hipGetLastError();
}

}  // namespace ivhd
