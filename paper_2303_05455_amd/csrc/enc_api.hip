// Host side of the parametric encoder ABI (include/ivhd.h, "parametric
// encoder"): an MLP n_in -> h1 -> h2 -> 2 with ReLU, BF16 weights and
// activations, FP32 accumulation and FP32 master weights, trained with Adam
// on the IVHD stress of its own batches' edges.
//
// One training step on a batch of R rows X_b (BF16):
//   H1 = relu(X_b W1^T + b1)  H2 = relu(H1 W2^T + b2)  Z = H2 W3^T + b3 (FP32)
//   loss = s E_batch(Z)       (the stress over the batch's local edge lists)
//   dZ   = grad E_batch(Z)    (the deterministic gather kernel of the loop)
//   dH2  = (dZ W3) . [H2 > 0]             dW3 = dZ^T H2      db3 = sum dZ
//   dH1  = (dH2 W2) . [H1 > 0]            dW2 = dH2^T H1     db2 = sum dH2
//                                         dW1 = dH1^T X_b    db1 = sum dH1
//   Adam on all parameters with the gradients scaled by s, then BF16 copies.
// The backward GEMMs read feature-major copies ([features][rows], rows
// padded to a multiple of 8 with zeros) of X_b, H1 and dH2 and produce dH1
// feature-major, so both operands of every GEMM are K-contiguous; db1 and
// db2 are row sums of those copies.
#include <cmath>
#include <mutex>
#include <new>
#include <unordered_set>

#include <algorithm>

#include "enc_internal.h"

struct ivhd_enc {
  int32_t n_in = 0, h1 = 0, h2 = 0;
  hipStream_t stream = nullptr;
  int64_t n_params = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *w16 = nullptr;
  int64_t t = 0;
  int64_t r_cap = 0;
  uint16_t *xb = nullptr, *a1 = nullptr, *a2 = nullptr, *d2 = nullptr;
  // feature-major copies [features][Rp] (Rp = rows rounded up to 8, the
  // padding zero) and W2 as [h1][h2], so that every backward GEMM reads both
  // operands with K contiguous; the layer-1 gradient exists only this way
  uint16_t *xbT = nullptr, *a1T = nullptr, *d1T = nullptr, *d2T = nullptr, *w2T = nullptr;
  float *z = nullptr, *dz = nullptr;
  float *ws = nullptr;
  int64_t ws_elems = 0;
  int splits = 32;   // K splits of the weight-gradient GEMMs: 8-14 output tiles each, so 256-448 blocks
  // epoch training state
  int32_t *rows = nullptr;
  int32_t *lnn = nullptr, *lrn = nullptr;
  ivhd_edges *plan = nullptr;
  int64_t plan_B = 0;
  int32_t plan_nn = 0, plan_rn = 0;
  int32_t *rn_all = nullptr;
  int64_t rn_all_elems = 0;
  int64_t *d_epoch = nullptr;
  double *d_losses = nullptr;
  int64_t losses_cap = 0;
};

using namespace ivhd;

namespace {

std::mutex g_enc_mu;
std::unordered_set<const ivhd_enc *> g_enc_live;

bool enc_live(const ivhd_enc *e) {
  if (!e) return false;
  std::lock_guard<std::mutex> lk(g_enc_mu);
  return g_enc_live.count(e) != 0;
}

void free_enc(ivhd_enc *e) {
  if (!e) return;
  if (e->plan) (void)ivhd_edges_destroy(e->plan);
  void *bufs[] = {e->w, e->g, e->m, e->v, e->w16, e->xb, e->a1, e->a2, e->d2, e->z, e->dz, e->ws,
                  e->rows, e->lnn, e->lrn, e->rn_all, e->d_epoch, e->d_losses, e->xbT, e->a1T, e->d1T, e->d2T,
                  e->w2T};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete e;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

GemmArgs gemm(const uint16_t *A, const uint16_t *B, int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb,
              void *C, int64_t ldc) {
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.vec_a = lda % 8 == 0 && aligned16(A);
  g.vec_b = ldb % 8 == 0 && aligned16(B);
  return g;
}

// forward of R rows (R <= r_cap) from BF16 input X (row pitch n_in) into z
int forward_rows(ivhd_enc *e, const uint16_t *X, int64_t R, float *z) {
  hipStream_t s = e->stream;
  GemmArgs g1 = gemm(X, e->w16 + e->oW1, R, e->h1, e->n_in, e->n_in, e->n_in, e->a1, e->h1);
  g1.bias = e->w + e->ob1;
  HIPCHK(launch_gemm_bf16(g1, 0, 1, GEMM_EPI_BIAS_RELU_BF16, 1, s));
  GemmArgs g2 = gemm(e->a1, e->w16 + e->oW2, R, e->h2, e->h1, e->h1, e->h1, e->a2, e->h2);
  g2.bias = e->w + e->ob2;
  HIPCHK(launch_gemm_bf16(g2, 0, 1, GEMM_EPI_BIAS_RELU_BF16, 1, s));
  HIPCHK(launch_head_forward(e->a2, R, e->h2, e->w16 + e->oW3, e->w + e->ob3, z, s));
  return IVHD_OK;
}

// weight gradient dW[M][N] = A^T B over R rows, split over K = R, into g;
// AT [M][R] and BT [N][R] are the transposed operands (K contiguous)
int wgrad(ivhd_enc *e, const uint16_t *AT, int64_t M, const uint16_t *BT, int64_t N, int64_t R, float *out) {
  hipStream_t s = e->stream;
  const int splits = gemm_splits_used(R, e->splits);
  GemmArgs gg = gemm(AT, BT, M, N, R, R, R, e->ws, N);
  HIPCHK(launch_gemm_bf16(gg, 0, 1, GEMM_EPI_F32, e->splits, s));
  HIPCHK(launch_splitk_reduce(e->ws, splits, M, N, N, out, N, s));
  return IVHD_OK;
}

// feature-major copy outT [C][Rp] of in [R][C] (16-byte tile path when it
// applies, else the element transposer)
int feature_major(const uint16_t *in, int64_t R, int64_t C, int64_t ldo, uint16_t *outT, hipStream_t s) {
  TileTArgs t;
  t.in = in;
  t.R = R;
  t.C = C;
  t.ldo = ldo;
  t.outT = outT;
  if (tile_t_ok(t)) {
    HIPCHK(launch_tile_t(TT_COPY, t, s));
  } else {
    HIPCHK(launch_transpose_bf16(in, R, C, outT, ldo, s));
  }
  return IVHD_OK;
}

// batch input rows into e->xb: rows[r] of src when rows is given, else the R
// rows of src; with the 16-byte path the feature-major copy e->xbT is
// written in the same pass (*xbT_ready)
int stage_batch(ivhd_enc *e, const uint16_t *src, const int32_t *rows, int64_t R, bool *xbT_ready) {
  hipStream_t s = e->stream;
  TileTArgs t;
  t.in = src;
  t.rows = rows;
  t.R = R;
  t.C = e->n_in;
  t.ldo = (R + 7) / 8 * 8;
  t.out = e->xb;
  t.outT = e->xbT;
  *xbT_ready = tile_t_ok(t);
  if (*xbT_ready) {
    HIPCHK(launch_tile_t(rows ? TT_GATHER : TT_COPY, t, s));
  } else if (rows) {
    HIPCHK(launch_gather_rows(src, e->n_in, rows, R, e->xb, s));
  } else {
    HIPCHK(hipMemcpyAsync(e->xb, src, (size_t)R * e->n_in * sizeof(uint16_t), hipMemcpyDeviceToDevice, s));
  }
  return IVHD_OK;
}

// one step on the batch already in e->xb (R rows) with local edge plan `plan`
int train_step_rows(ivhd_enc *e, int64_t R, bool xbT_ready, ivhd_edges *plan, float c, float eps, float lr,
                    float scale, double *d_loss) {
  hipStream_t s = e->stream;
  const int64_t Rp = (R + 7) / 8 * 8;
  int rc = forward_rows(e, e->xb, R, e->z);
  if (rc) return rc;
  if (!xbT_ready && (rc = feature_major(e->xb, R, e->n_in, Rp, e->xbT, s))) return rc;
  if ((rc = feature_major(e->a1, R, e->h1, Rp, e->a1T, s))) return rc;
  if ((rc = feature_major(e->w16 + e->oW2, e->h2, e->h1, e->h2, e->w2T, s))) return rc;
  if (d_loss) {   // the batch stress and its gradient from one pass
    if ((rc = ivhd_edges_stress_grad(plan, e->z, c, eps, nullptr, d_loss, e->dz))) return rc;
  } else if ((rc = ivhd_edges_grad(plan, e->z, c, eps, nullptr, e->dz))) {
    return rc;
  }
  // head: d2 = input gradient of the head, row-major and feature-major
  TileTArgs hd;
  hd.in = e->a2;
  hd.dz = e->dz;
  hd.w3 = e->w16 + e->oW3;
  hd.R = R;
  hd.C = e->h2;
  hd.ldo = Rp;
  hd.out = e->d2;
  hd.outT = e->d2T;
  if (tile_t_ok(hd)) {
    HIPCHK(launch_tile_t(TT_HEAD_DGRAD, hd, s));
  } else {
    HIPCHK(launch_head_dgrad(e->dz, e->w16 + e->oW3, e->a2, R, e->h2, e->d2, s));
    HIPCHK(launch_transpose_bf16(e->d2, R, e->h2, e->d2T, Rp, s));
  }
  HIPCHK(launch_colsum(1, e->a2, e->dz, R, 2 * (int64_t)e->h2, e->h2, e->ws, e->g + e->oW3, s));
  HIPCHK(launch_colsum(2, e->dz, nullptr, R, 2, 2, e->ws, e->g + e->ob3, s));
  HIPCHK(launch_rowsum_bf16(e->d2T, e->h2, Rp, e->g + e->ob2, s));
  // layer 2, feature-major: d1^T = (W2^T d2^T) * relu'(a1^T); columns r >= R
  // come out zero because the mask a1^T is zero there (rows of d2 past R are
  // never multiplied into a stored value otherwise)
  GemmArgs gd = gemm(e->w2T, e->d2, e->h1, Rp, e->h2, e->h2, e->h2, e->d1T, Rp);
  gd.mask = e->a1T;
  gd.ldm = Rp;
  HIPCHK(launch_gemm_bf16(gd, 0, 1, GEMM_EPI_RELU_MASK_BF16, 1, s));
  if ((rc = wgrad(e, e->d2T, e->h2, e->a1T, e->h1, Rp, e->g + e->oW2))) return rc;
  // layer 1
  HIPCHK(launch_rowsum_bf16(e->d1T, e->h1, Rp, e->g + e->ob1, s));
  if ((rc = wgrad(e, e->d1T, e->h1, e->xbT, e->n_in, Rp, e->g + e->oW1))) return rc;
  // Adam
  e->t += 1;
  HIPCHK(launch_adam(e->w, e->g, e->m, e->v, e->w16, e->n_params, lr, 0.9f, 0.999f, 1e-8f, e->t, scale, s));
  return IVHD_OK;
}

uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

extern "C" {

int ivhd_enc_create(ivhd_enc **out, int32_t n_in, int32_t h1, int32_t h2, uint64_t seed, int64_t max_rows,
                    void *stream) {
  clear_error();
  if (!out) return fail(IVHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || h1 < 1 || h2 < 1 || n_in > 65536 || h1 > 65536 || h2 > 65536)
    return fail(IVHD_EINVAL, "layer widths (%d, %d, %d) outside [1, 65536]", n_in, h1, h2);
  if (h1 % 8 || h2 % 8) return fail(IVHD_EINVAL, "hidden widths (%d, %d) must be multiples of 8", h1, h2);
  if (max_rows < 1 || max_rows > (int64_t)1 << 26)
    return fail(IVHD_EINVAL, "max_rows = %lld outside [1, 2^26]", (long long)max_rows);
  ivhd_enc *e = new (std::nothrow) ivhd_enc();
  if (!e) return fail(IVHD_ENOMEM, "host allocation of the encoder failed");
  e->n_in = n_in;
  e->h1 = h1;
  e->h2 = h2;
  e->stream = (hipStream_t)stream;
  e->oW1 = 0;
  e->ob1 = e->oW1 + (int64_t)h1 * n_in;
  e->oW2 = e->ob1 + h1;
  e->ob2 = e->oW2 + (int64_t)h2 * h1;
  e->oW3 = e->ob2 + h2;
  e->ob3 = e->oW3 + 2 * (int64_t)h2;
  e->n_params = e->ob3 + 2;
  e->r_cap = max_rows;
  const int64_t wmax = (int64_t)h1 * n_in > (int64_t)h2 * h1 ? (int64_t)h1 * n_in : (int64_t)h2 * h1;
  e->ws_elems = wmax * e->splits;
  const int64_t jmax = std::max<int64_t>(2 * (int64_t)h2, std::max(h1, h2));
  const int64_t colsum_ws = colsum_workspace(max_rows, jmax);
  if (colsum_ws > e->ws_elems) e->ws_elems = colsum_ws;
  int rc;
#define ENC_CHK(expr) \
  do {                \
    rc = (expr);      \
    if (rc) {         \
      free_enc(e);    \
      return rc;      \
    }                 \
  } while (0)
#define ENC_HIP(expr)                 \
  do {                                \
    hipError_t _e = (expr);           \
    if (_e != hipSuccess) {           \
      rc = hip_fail(_e, #expr);       \
      free_enc(e);                    \
      return rc;                      \
    }                                 \
  } while (0)
  const int64_t np = e->n_params;
  ENC_CHK(dev_alloc(&e->w, np, "encoder weights"));
  ENC_CHK(dev_alloc(&e->g, np, "encoder gradients"));
  ENC_CHK(dev_alloc(&e->m, np, "Adam first moments"));
  ENC_CHK(dev_alloc(&e->v, np, "Adam second moments"));
  ENC_CHK(dev_alloc(&e->w16, np, "BF16 weights"));
  ENC_CHK(dev_alloc(&e->xb, max_rows * n_in, "batch input"));
  ENC_CHK(dev_alloc(&e->a1, max_rows * h1, "layer-1 activations"));
  ENC_CHK(dev_alloc(&e->a2, max_rows * h2, "layer-2 activations"));
  const int64_t rows_p = (max_rows + 7) / 8 * 8;
  // read as a GEMM operand of Rp rows
  ENC_CHK(dev_alloc(&e->d2, rows_p * h2, "layer-2 gradients"));
  ENC_CHK(dev_alloc(&e->xbT, rows_p * n_in, "feature-major batch input"));
  ENC_CHK(dev_alloc(&e->a1T, rows_p * h1, "feature-major layer-1 activations"));
  ENC_CHK(dev_alloc(&e->d1T, rows_p * h1, "feature-major layer-1 gradients"));
  ENC_CHK(dev_alloc(&e->d2T, rows_p * h2, "feature-major layer-2 gradients"));
  ENC_CHK(dev_alloc(&e->w2T, (int64_t)h1 * h2, "transposed W2"));
  ENC_CHK(dev_alloc(&e->z, max_rows * 2, "embedding"));
  ENC_CHK(dev_alloc(&e->dz, max_rows * 2, "embedding gradient"));
  ENC_CHK(dev_alloc(&e->ws, e->ws_elems, "encoder workspace"));
  ENC_CHK(dev_alloc(&e->d_epoch, 1, "epoch counter"));
  hipStream_t s = e->stream;
  ENC_HIP(launch_fill_i32((int32_t *)e->w, np, 0, s));
  ENC_HIP(launch_fill_i32((int32_t *)e->m, np, 0, s));
  ENC_HIP(launch_fill_i32((int32_t *)e->v, np, 0, s));
  ENC_HIP(launch_fill_i32((int32_t *)e->g, np, 0, s));
  ENC_HIP(launch_glorot(e->w + e->oW1, (int64_t)h1 * n_in, n_in, h1, seed, 1, s));
  ENC_HIP(launch_glorot(e->w + e->oW2, (int64_t)h2 * h1, h1, h2, seed, 2ull << 40, s));
  ENC_HIP(launch_glorot(e->w + e->oW3, 2 * (int64_t)h2, h2, 2, seed, 3ull << 40, s));
  ENC_HIP(launch_f32_to_bf16(e->w, np, e->w16, s));
  ENC_HIP(hipStreamSynchronize(s));
#undef ENC_CHK
#undef ENC_HIP
  {
    std::lock_guard<std::mutex> lk(g_enc_mu);
    g_enc_live.insert(e);
  }
  *out = e;
  return IVHD_OK;
}

int ivhd_enc_num_params(const ivhd_enc *e, int64_t *h_n) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  if (!h_n) return fail(IVHD_EINVAL, "h_n is NULL");
  *h_n = e->n_params;
  return IVHD_OK;
}

int ivhd_enc_get_params(ivhd_enc *e, float *d_params, float *d_grads) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  const size_t bytes = (size_t)e->n_params * sizeof(float);
  if (d_params) HIPCHK(hipMemcpyAsync(d_params, e->w, bytes, hipMemcpyDeviceToDevice, e->stream));
  if (d_grads) HIPCHK(hipMemcpyAsync(d_grads, e->g, bytes, hipMemcpyDeviceToDevice, e->stream));
  return IVHD_OK;
}

int ivhd_enc_set_params(ivhd_enc *e, const float *d_params) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  if (!d_params) return fail(IVHD_EINVAL, "d_params is NULL");
  HIPCHK(hipMemcpyAsync(e->w, d_params, (size_t)e->n_params * sizeof(float), hipMemcpyDeviceToDevice, e->stream));
  HIPCHK(launch_f32_to_bf16(e->w, e->n_params, e->w16, e->stream));
  HIPCHK(launch_fill_i32((int32_t *)e->m, e->n_params, 0, e->stream));
  HIPCHK(launch_fill_i32((int32_t *)e->v, e->n_params, 0, e->stream));
  e->t = 0;
  return IVHD_OK;
}

int ivhd_enc_embed(ivhd_enc *e, const uint16_t *d_x16, int64_t rows, float *d_z) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  if (rows < 0) return fail(IVHD_EINVAL, "rows = %lld < 0", (long long)rows);
  if (rows > 0 && (!d_x16 || !d_z)) return fail(IVHD_EINVAL, "d_x16 and d_z must not be NULL");
  for (int64_t r0 = 0; r0 < rows; r0 += e->r_cap) {
    const int64_t R = rows - r0 < e->r_cap ? rows - r0 : e->r_cap;
    int rc = forward_rows(e, d_x16 + r0 * e->n_in, R, d_z + 2 * r0);
    if (rc) return rc;
  }
  return IVHD_OK;
}

int ivhd_enc_train_step(ivhd_enc *e, const uint16_t *d_xb16, int64_t R, ivhd_edges *plan, float c, float eps,
                        float lr, float loss_scale, double *d_loss) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  if (R < 1 || R > e->r_cap) return fail(IVHD_EINVAL, "R = %lld outside [1, max_rows]", (long long)R);
  if (!d_xb16 || !plan) return fail(IVHD_EINVAL, "d_xb16 and plan must not be NULL");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(IVHD_EINVAL, "lr = %g must be > 0", (double)lr);
  bool ready = false;
  int rc = stage_batch(e, d_xb16, nullptr, R, &ready);
  if (rc) return rc;
  return train_step_rows(e, R, ready, plan, c, eps, lr, loss_scale, d_loss);
}

int ivhd_enc_train_epoch(ivhd_enc *e, const uint16_t *d_x16, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                         int32_t rn, uint64_t seed, int64_t epoch, int64_t batch, float c, float eps, float lr,
                         double *h_loss) {
  if (!enc_live(e)) return fail(IVHD_ESTATE, "invalid encoder");
  if (!d_x16 || !d_nn_idx) return fail(IVHD_EINVAL, "d_x16 and d_nn_idx must not be NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (nn < 1 || nn > 64 || rn < 0 || rn > 64 || nn + rn > M - 1)
    return fail(IVHD_EINVAL, "nn = %d, rn = %d invalid for M = %lld", nn, rn, (long long)M);
  if (batch < 1 || batch * (1 + nn + rn) > e->r_cap)
    return fail(IVHD_EINVAL, "batch = %lld: batch * (1 + nn + rn) must be in [1, max_rows]", (long long)batch);
  if (epoch < 0) return fail(IVHD_EINVAL, "epoch = %lld < 0", (long long)epoch);
  hipStream_t s = e->stream;
  const int64_t R = batch * (1 + nn + rn);
  int rc;
  // local edge lists of a batch: fixed structure, built once per (batch, nn, rn)
  if (!e->plan || e->plan_B != batch || e->plan_nn != nn || e->plan_rn != rn) {
    if (e->plan) {
      (void)ivhd_edges_destroy(e->plan);
      e->plan = nullptr;
    }
    if (e->lnn) (void)hipFree(e->lnn);
    if (e->lrn) (void)hipFree(e->lrn);
    if (e->rows) (void)hipFree(e->rows);
    e->lnn = e->lrn = e->rows = nullptr;
    if ((rc = dev_alloc(&e->lnn, R * nn, "batch nn lists"))) return rc;
    if (rn > 0 && (rc = dev_alloc(&e->lrn, R * rn, "batch rn lists"))) return rc;
    if ((rc = dev_alloc(&e->rows, R, "batch rows"))) return rc;
    HIPCHK(launch_batch_plan(batch, nn, rn, e->lnn, e->lrn, s));
    if ((rc = ivhd_edges_create(&e->plan, R, e->lnn, nn, e->lrn, rn, 0, s))) return rc;
    e->plan_B = batch;
    e->plan_nn = nn;
    e->plan_rn = rn;
  }
  if (rn > 0 && e->rn_all_elems < M * rn) {
    if (e->rn_all) (void)hipFree(e->rn_all);
    e->rn_all = nullptr;
    e->rn_all_elems = 0;
    if ((rc = dev_alloc(&e->rn_all, M * rn, "epoch random neighbours"))) return rc;
    e->rn_all_elems = M * rn;
  }
  const int64_t steps = (M + batch - 1) / batch;
  if (e->losses_cap < steps) {
    if (e->d_losses) (void)hipFree(e->d_losses);
    e->d_losses = nullptr;
    e->losses_cap = 0;
    if ((rc = dev_alloc(&e->d_losses, steps, "step losses"))) return rc;
    e->losses_cap = steps;
  }
  // the epoch's random neighbours (same draw as the loop's, epoch = training epoch)
  if (rn > 0) {
    HIPCHK(hipMemcpyAsync(e->d_epoch, &epoch, sizeof epoch, hipMemcpyHostToDevice, s));
    HIPCHK(launch_rn_sample(d_nn_idx, M, nn, rn, seed, e->d_epoch, nullptr, nullptr, e->rn_all, nullptr, nullptr, s));
    HIPCHK(hipStreamSynchronize(s));   // epoch lives on the host stack
  }
  // visiting order: s_b = (a b + c0) mod M with gcd(a, M) = 1, a bijection
  uint64_t a = mix64(seed ^ mix64(0x5eedULL + (uint64_t)epoch)) % (uint64_t)M;
  if (a == 0) a = 1;
  while (gcd64(a, (uint64_t)M) != 1) a = a + 1 == (uint64_t)M ? 1 : a + 1;
  const uint64_t c0 = mix64(seed + 7919ull * (uint64_t)epoch) % (uint64_t)M;
  const float scale = 1.f / (float)batch;
  for (int64_t st = 0; st < steps; ++st) {
    HIPCHK(launch_batch_rows(d_nn_idx, nn, e->rn_all, rn, M, batch, a, c0, st * batch, e->rows, s));
    bool ready = false;
    if ((rc = stage_batch(e, d_x16, e->rows, R, &ready))) return rc;
    if ((rc = train_step_rows(e, R, ready, e->plan, c, eps, lr, scale, e->d_losses + st))) return rc;
  }
  if (h_loss) {
    double *tmp = new (std::nothrow) double[steps];
    if (!tmp) return fail(IVHD_ENOMEM, "host loss buffer");
    hipError_t err = hipMemcpyAsync(tmp, e->d_losses, steps * sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    double sum = 0.0;
    for (int64_t st = 0; st < steps; ++st) sum += tmp[st];
    delete[] tmp;
    if (err != hipSuccess) return hip_fail(err, "loss copy");
    *h_loss = sum * scale / (double)steps;
  }
  return IVHD_OK;
}

int ivhd_enc_destroy(ivhd_enc *e) {
  if (!e) return IVHD_OK;
  {
    std::lock_guard<std::mutex> lk(g_enc_mu);
    if (!g_enc_live.erase(e)) return fail(IVHD_ESTATE, "invalid encoder");
  }
  hipError_t err = hipStreamSynchronize(e->stream);
  free_enc(e);
  if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
  return IVHD_OK;
}

int ivhd_f32_to_bf16(const float *d_x, int64_t n, uint16_t *d_y, void *stream) {
  if (n < 0) return fail(IVHD_EINVAL, "n < 0");
  if (n > 0 && (!d_x || !d_y)) return fail(IVHD_EINVAL, "d_x and d_y must not be NULL");
  if (n == 0) return IVHD_OK;
  HIPCHK(launch_f32_to_bf16(d_x, n, d_y, (hipStream_t)stream));
  return IVHD_OK;
}

int ivhd_gemm_bf16(const uint16_t *d_a, const uint16_t *d_b, int64_t M, int64_t N, int64_t K, int64_t lda,
                   int64_t ldb, int32_t trans_a, int32_t trans_b, int32_t epilogue, const float *d_bias,
                   const uint16_t *d_mask, int64_t ldm, void *d_c, int64_t ldc, int32_t splits, float *d_work,
                   void *stream) {
  if (!d_a || !d_b || !d_c) return fail(IVHD_EINVAL, "d_a, d_b and d_c must not be NULL");
  if (M < 1 || N < 1 || K < 1) return fail(IVHD_EINVAL, "M, N, K must be >= 1");
  if (epilogue < 0 || epilogue > 2) return fail(IVHD_EINVAL, "epilogue = %d unknown", epilogue);
  if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N) || ldc < N)
    return fail(IVHD_EINVAL, "leading dimension too small");
  if (epilogue == 2 && (!d_mask || ldm < N)) return fail(IVHD_EINVAL, "epilogue 2 needs d_mask with ldm >= N");
  if (splits < 1) splits = 1;
  const int used = gemm_splits_used(K, splits);
  if (used > 1 && (epilogue != 0 || !d_work)) return fail(IVHD_EINVAL, "split-K needs epilogue 0 and d_work");
  hipStream_t s = (hipStream_t)stream;
  GemmArgs g = gemm(d_a, d_b, M, N, K, lda, ldb, used > 1 ? (void *)d_work : d_c, used > 1 ? N : ldc);
  g.bias = d_bias;
  g.mask = d_mask;
  g.ldm = ldm;
  HIPCHK(launch_gemm_bf16(g, trans_a ? 1 : 0, trans_b ? 1 : 0, epilogue, splits, s));
  if (used > 1) HIPCHK(launch_splitk_reduce(d_work, used, M, N, N, (float *)d_c, ldc, s));
  return IVHD_OK;
}

}  // extern "C"
