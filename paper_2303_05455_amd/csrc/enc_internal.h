// Internal declarations of the encoder kernels (enc.hip) and host code
// (enc_api.hip).  Not part of the public ABI.
#pragma once

#include "ivhd_internal.h"

namespace ivhd {

enum { GEMM_EPI_F32 = 0, GEMM_EPI_BIAS_RELU_BF16 = 1, GEMM_EPI_RELU_MASK_BF16 = 2 };

struct GemmArgs {
  const uint16_t *A;
  const uint16_t *B;
  int64_t M, N, K;
  int64_t lda, ldb;
  int64_t kchunk;          // K range per blockIdx.z (set by launch_gemm_bf16)
  const float *bias;       // [N] or NULL (GEMM_EPI_BIAS_RELU_BF16)
  const uint16_t *mask;    // [M][ldm] forward activation (GEMM_EPI_RELU_MASK_BF16)
  int64_t ldm;
  void *C;                 // FP32 slabs [splits][M][ldc] or BF16 [M][ldc]
  int64_t ldc;
  bool vec_a, vec_b;       // 16-byte vector loads allowed (ld % 8 == 0, aligned base)
};

hipError_t launch_gemm_bf16(const GemmArgs &g, int ta, int tb, int epi, int splits, hipStream_t s);
int gemm_splits_used(int64_t K, int splits);
hipError_t launch_splitk_reduce(const float *part, int splits, int64_t M, int64_t N, int64_t ldp, float *out,
                                int64_t ldo, hipStream_t s);
hipError_t launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s);
hipError_t launch_gather_rows(const uint16_t *X, int64_t N, const int32_t *rows, int64_t R, uint16_t *out,
                              hipStream_t s);
hipError_t launch_head_forward(const uint16_t *H, int64_t R, int K, const uint16_t *W3, const float *b3, float *Z,
                               hipStream_t s);
hipError_t launch_head_dgrad(const float *dZ, const uint16_t *W3, const uint16_t *H, int64_t R, int K,
                             uint16_t *dH, hipStream_t s);
// column sums over R rows as a fixed-order tree of kColsumRows-row partial
// sums (deterministic); see colsum_kernel for the modes.  ws must hold
// colsum_workspace(R, J) floats.
constexpr int kColsumRows = 256;
int64_t colsum_workspace(int64_t R, int64_t J);
// out [C][ldo] = transpose of the BF16 matrix in [R][C], entries r >= R of
// each out row zero (ldo >= R)
hipError_t launch_transpose_bf16(const uint16_t *in, int64_t R, int64_t C, uint16_t *out, int64_t ldo,
                                 hipStream_t s);
// tile transposer with a fused producer (see tile_t_kernel for the modes)
enum { TT_COPY = 0, TT_GATHER = 1, TT_HEAD_DGRAD = 2 };
struct TileTArgs {
  const uint16_t *in = nullptr;     // [R][C] (TT_GATHER: the data, rows[r] selects)
  const int32_t *rows = nullptr;    // TT_GATHER
  const float *dz = nullptr;        // TT_HEAD_DGRAD: [R][2]
  const uint16_t *w3 = nullptr;     // TT_HEAD_DGRAD: [2][C]
  int64_t R = 0, C = 0, ldo = 0;
  uint16_t *out = nullptr;          // [R][C] row-major copy, or NULL
  uint16_t *outT = nullptr;         // [C][ldo]
};
bool tile_t_ok(const TileTArgs &a);
hipError_t launch_tile_t(int mode, const TileTArgs &a, hipStream_t s);
// out[j] = sum of row j of the BF16 matrix X [J][L] (fixed order)
hipError_t launch_rowsum_bf16(const uint16_t *X, int64_t J, int64_t L, float *out, hipStream_t s);
hipError_t launch_colsum(int mode, const void *X, const float *dZ, int64_t R, int64_t J, int64_t K, float *ws,
                         float *out, hipStream_t s);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, uint16_t *w16, int64_t n, float lr, float b1,
                       float b2, float eps, int64_t t, float gscale, hipStream_t s);
hipError_t launch_glorot(float *w, int64_t n, int fan_in, int fan_out, uint64_t seed, uint64_t offset,
                         hipStream_t s);

hipError_t launch_batch_rows(const int32_t *nn_idx, int nn, const int32_t *rn_idx, int rn, int64_t M, int64_t B,
                             uint64_t a, uint64_t c0, int64_t off, int32_t *rows, hipStream_t s);
hipError_t launch_batch_plan(int64_t B, int nn, int rn, int32_t *lnn, int32_t *lrn, hipStream_t s);

}  // namespace ivhd
