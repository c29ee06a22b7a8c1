// Host side of the C ABI declared in include/ivhd.h: argument validation,
// context lifetime, the random-neighbour epochs, the ping-pong of the
// positions and the HIP-graph replay of the iteration loop.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>

#include "ivhd_internal.h"

using namespace ivhd;

namespace ivhd {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? IVHD_ENOMEM : IVHD_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

}  // namespace ivhd

namespace {

// contexts handed out and not yet destroyed: a stale or foreign pointer is
// reported as IVHD_ESTATE instead of being dereferenced
std::mutex g_live_mu;
std::unordered_set<const ivhd_ctx *> g_live;

constexpr int kChunkIters = 64;            // graph length when random neighbours are drawn once

}  // namespace

struct ivhd_ctx {
  ivhd_params p{};
  hipStream_t stream = nullptr;   // caller's
  hipStream_t cap = nullptr;      // private stream used only for graph capture
  const int32_t *nn_idx = nullptr;
  float2 *y_user = nullptr, *v = nullptr, *y_alt = nullptr;
  int parity = 0;                 // det mode: 0 -> Y_n in y_user, 1 -> in y_alt
  Csc nn_csc, rn_csc;
  CscScratch sc;
  int32_t *rn_idx = nullptr;
  int64_t *epoch = nullptr;
  int32_t *flags = nullptr;
  float2 *fbuf = nullptr;
  int32_t *heavy = nullptr;       // vertices served by a whole wavefront (det mode)
  int32_t n_heavy = 0;
  double *partials = nullptr;
  int nparts = 0;
  double *d_E = nullptr;
  int64_t n = 0;
  int use_graphs = 1;
  hipGraphExec_t g_epoch[2] = {nullptr, nullptr};   // draw + R iterations
  hipGraphExec_t g_first[2] = {nullptr, nullptr};   // the R iterations of epoch 0
  hipGraphExec_t g_chunk[2] = {nullptr, nullptr};   // kChunkIters iterations (no draws)

  bool det() const { return p.mode == IVHD_MODE_DET; }
  float2 *cur() const { return parity ? y_alt : y_user; }
  float2 *other() const { return parity ? y_user : y_alt; }
};

namespace {

void free_ctx(ivhd_ctx *c) {
  if (!c) return;
  for (int k = 0; k < 2; ++k) {
    if (c->g_epoch[k]) (void)hipGraphExecDestroy(c->g_epoch[k]);
    if (c->g_first[k]) (void)hipGraphExecDestroy(c->g_first[k]);
    if (c->g_chunk[k]) (void)hipGraphExecDestroy(c->g_chunk[k]);
  }
  void *bufs[] = {c->y_alt, c->nn_csc.ptr, c->nn_csc.src, c->rn_csc.ptr, c->rn_csc.src,
                  c->sc.cnt, c->sc.tmp, c->sc.part, c->sc.big, c->rn_idx, c->epoch,
                  c->flags, c->fbuf, c->heavy, c->partials, c->d_E};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

bool live(const ivhd_ctx *c) {
  if (!c) return false;
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(c) != 0;
}

int validate(const ivhd_params *p) {
  if (!p) return fail(IVHD_EINVAL, "params is NULL");
  if (p->M < 2 || p->M > (int64_t)INT32_MAX - 1)
    return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)p->M);
  if (p->nn < 1 || p->nn > 64) return fail(IVHD_EINVAL, "nn = %d outside [1, 64]", p->nn);
  if (p->rn < 0 || p->rn > 64) return fail(IVHD_EINVAL, "rn = %d outside [0, 64]", p->rn);
  if ((int64_t)p->nn + p->rn > p->M - 1)
    return fail(IVHD_EINVAL, "nn + rn = %d exceeds M - 1 = %lld", p->nn + p->rn,
                (long long)(p->M - 1));
  if (p->M * (int64_t)(p->nn > p->rn ? p->nn : p->rn) > (int64_t)INT32_MAX)
    return fail(IVHD_EINVAL, "M * max(nn, rn) exceeds 2^31-1 edges");
  if (!std::isfinite(p->a) || p->a < 0.f || p->a > 1.f)
    return fail(IVHD_EINVAL, "a = %g outside [0, 1]", (double)p->a);
  if (!std::isfinite(p->b) || !(p->b > 0.f)) return fail(IVHD_EINVAL, "b = %g must be > 0", (double)p->b);
  if (!std::isfinite(p->c) || !(p->c > 0.f) || !(p->c < 1.f))
    return fail(IVHD_EINVAL, "c = %g outside (0, 1)", (double)p->c);
  if (!std::isfinite(p->eps) || p->eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)p->eps);
  if (p->rn_resample_every < 0)
    return fail(IVHD_EINVAL, "rn_resample_every = %d must be >= 0", p->rn_resample_every);
  if (p->mode != IVHD_MODE_DET && p->mode != IVHD_MODE_ATOMIC)
    return fail(IVHD_EINVAL, "mode = %d is neither IVHD_MODE_DET nor IVHD_MODE_ATOMIC", p->mode);
  return IVHD_OK;
}

StepArgs step_args(const ivhd_ctx *c, const float2 *y, float2 *y_out) {
  StepArgs a;
  a.y = y;
  a.y_out = y_out;
  a.v = c->v;
  a.nn_idx = c->nn_idx;
  a.rn_idx = c->rn_idx;
  a.nn_ptr = c->nn_csc.ptr;
  a.nn_src = c->nn_csc.src;
  a.rn_ptr = c->rn_csc.ptr;
  a.rn_src = c->rn_csc.src;
  a.fbuf = c->fbuf;
  a.flags = c->flags;
  a.gscale = nullptr;
  a.heavy = c->heavy;
  a.n_heavy = c->n_heavy;
  a.heavy_blocks = (c->n_heavy + kHeavyPerBlock - 1) / kHeavyPerBlock;
  a.M = c->p.M;
  a.nn = c->p.nn;
  a.rn = c->p.rn;
  a.a = c->p.a;
  a.b = c->p.b;
  a.c = c->p.c;
  a.eps = c->p.eps;
  return a;
}

// A new random-neighbour epoch: epoch += 1, draw, and (det mode) rebuild the
// transposed rn lists.
int enqueue_draw(ivhd_ctx *c, hipStream_t s) {
  if (c->p.rn == 0) return IVHD_OK;
  const int64_t M = c->p.M;
  int32_t *cnt = c->det() ? c->sc.cnt : nullptr;
  HIPCHK(launch_epoch_begin(c->epoch, cnt, M, c->flags, s));
  HIPCHK(launch_rn_sample(c->nn_idx, M, c->p.nn, c->p.rn, c->p.seed, c->epoch, c->rn_idx, cnt, s));
  if (c->det()) {
    HIPCHK(launch_scan(c->sc.cnt, M, c->sc.part, c->rn_csc.ptr, s));
    HIPCHK(launch_scatter_sort(c->rn_idx, M, c->p.rn, c->rn_csc.ptr, c->sc.cnt, c->sc.tmp,
                               c->sc.big, c->flags, c->rn_csc.src, s));
  }
  return IVHD_OK;
}

// `count` iterations starting from parity `par`; returns the final parity.
int enqueue_steps(ivhd_ctx *c, hipStream_t s, int64_t count, int *par) {
  for (int64_t k = 0; k < count; ++k) {
    if (c->det()) {
      float2 *src = *par ? c->y_alt : c->y_user;
      float2 *dst = *par ? c->y_user : c->y_alt;
      HIPCHK(launch_step_det(step_args(c, src, dst), s));
      *par ^= 1;
    } else {
      HIPCHK(launch_step_atomic(step_args(c, c->y_user, c->y_user), s));
    }
  }
  return IVHD_OK;
}

int capture(ivhd_ctx *c, bool with_draw, int64_t count, int par, hipGraphExec_t *out) {
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int rc = with_draw ? enqueue_draw(c, c->cap) : IVHD_OK;
  int p = par;
  if (rc == IVHD_OK) rc = enqueue_steps(c, c->cap, count, &p);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc != IVHD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return IVHD_OK;
}

// transposed lists of an [M][k] index list into g (sources ascending per target)
int build_csc(const int32_t *idx, int64_t M, int k, Csc &g, CscScratch &sc, int32_t *flags,
              hipStream_t s) {
  HIPCHK(launch_fill_i32(sc.cnt, M + 1, 0, s));
  HIPCHK(launch_fill_i32(flags + FLAG_BIG_COUNT, 1, 0, s));
  HIPCHK(launch_count(idx, M, k, sc.cnt, s));
  HIPCHK(launch_scan(sc.cnt, M, sc.part, g.ptr, s));
  HIPCHK(launch_scatter_sort(idx, M, k, g.ptr, sc.cnt, sc.tmp, sc.big, flags, g.src, s));
  return IVHD_OK;
}

// the vertices of nn in-degree above kHeavyDegree; synchronises s to read the count
int build_heavy(const Csc &nn_csc, int64_t M, int32_t *heavy, int32_t *flags, int32_t *n_heavy,
                hipStream_t s) {
  HIPCHK(launch_fill_i32(flags + FLAG_BIG_COUNT, 1, 0, s));
  HIPCHK(launch_heavy_list(nn_csc.ptr, M, heavy, flags + FLAG_BIG_COUNT, s));
  HIPCHK(hipMemcpyAsync(n_heavy, flags + FLAG_BIG_COUNT, sizeof *n_heavy, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return IVHD_OK;
}

int build_nn_csc(ivhd_ctx *c) {
  return build_csc(c->nn_idx, c->p.M, c->p.nn, c->nn_csc, c->sc, c->flags, c->stream);
}

}  // namespace

extern "C" {

const char *ivhd_last_error(void) { return ivhd::g_err.c_str(); }

int ivhd_version(void) { return 100; }

int ivhd_init(ivhd_ctx **out, const ivhd_params *p, const int32_t *d_nn_idx, float *d_y,
              float *d_v, void *stream) {
  clear_error();
  if (!out) return fail(IVHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!d_nn_idx) return fail(IVHD_EINVAL, "d_nn_idx is NULL");
  if (!d_y) return fail(IVHD_EINVAL, "d_y is NULL");
  if (!d_v) return fail(IVHD_EINVAL, "d_v is NULL");
  if (d_y == d_v) return fail(IVHD_EINVAL, "d_y and d_v alias");

  ivhd_ctx *c = new (std::nothrow) ivhd_ctx();
  if (!c) return fail(IVHD_ENOMEM, "host allocation of the context failed");
  c->p = *p;
  c->stream = (hipStream_t)stream;
  c->nn_idx = d_nn_idx;
  c->y_user = (float2 *)d_y;
  c->v = (float2 *)d_v;
  const int64_t M = p->M;
  const int64_t nb = (M + kScanChunk - 1) / kScanChunk;
  const int64_t cap_tmp = M * (int64_t)(p->nn > p->rn ? p->nn : p->rn);

#define ALLOC(ptr, n, what)                    \
  do {                                         \
    rc = dev_alloc(&(ptr), (size_t)(n), what); \
    if (rc) {                                  \
      free_ctx(c);                             \
      return rc;                               \
    }                                          \
  } while (0)
#define CHK(expr)      \
  do {                 \
    rc = (expr);       \
    if (rc) {          \
      free_ctx(c);     \
      return rc;       \
    }                  \
  } while (0)
#define HIPCHK_C(expr)                                  \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) {                             \
      rc = hip_fail(_e, #expr);                         \
      free_ctx(c);                                      \
      return rc;                                        \
    }                                                   \
  } while (0)

  HIPCHK_C(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  if (p->mode == IVHD_MODE_DET) ALLOC(c->y_alt, M, "the second position buffer");
  ALLOC(c->nn_csc.ptr, M + 1, "nn in-edge offsets");
  ALLOC(c->nn_csc.src, M * p->nn, "nn in-edge sources");
  ALLOC(c->sc.cnt, M + 1, "CSC counts");
  ALLOC(c->sc.tmp, cap_tmp, "CSC scatter buffer");
  ALLOC(c->sc.part, nb + 1, "scan partials");
  ALLOC(c->sc.big, M, "large-segment list");
  ALLOC(c->epoch, 1, "epoch counter");
  ALLOC(c->flags, FLAG_SLOTS, "device flags");
  if (p->rn > 0) {
    ALLOC(c->rn_idx, M * p->rn, "random neighbours");
    if (p->mode == IVHD_MODE_DET) {
      ALLOC(c->rn_csc.ptr, M + 1, "rn in-edge offsets");
      ALLOC(c->rn_csc.src, M * p->rn, "rn in-edge sources");
    }
  }
  if (p->mode == IVHD_MODE_ATOMIC) ALLOC(c->fbuf, M, "force accumulator");
  if (p->mode == IVHD_MODE_DET) ALLOC(c->heavy, M, "heavy-vertex list");
  c->nparts = stress_partials(M);
  ALLOC(c->partials, c->nparts, "stress partials");
  ALLOC(c->d_E, 1, "stress result");

  hipStream_t s = c->stream;
  HIPCHK_C(launch_fill_i32(c->flags, FLAG_SLOTS, 0, s));
  HIPCHK_C(launch_validate_idx(d_nn_idx, M, p->nn, -1, c->flags, s));
  int32_t hflags[FLAG_SLOTS];
  HIPCHK_C(hipMemcpyAsync(hflags, c->flags, sizeof hflags, hipMemcpyDeviceToHost, s));
  HIPCHK_C(hipStreamSynchronize(s));
  if (hflags[FLAG_BAD_INDEX]) {
    free_ctx(c);
    return fail(IVHD_EINVAL, "nn_idx holds an entry outside [-1, M) or a self edge");
  }
  CHK(build_nn_csc(c));
  if (c->heavy) CHK(build_heavy(c->nn_csc, M, c->heavy, c->flags, &c->n_heavy, s));
  if (c->fbuf) HIPCHK_C(launch_fill_i32((int32_t *)c->fbuf, 2 * M, 0, s));
  const int64_t minus_one = -1;
  HIPCHK_C(hipMemcpyAsync(c->epoch, &minus_one, sizeof minus_one, hipMemcpyHostToDevice, s));
  CHK(enqueue_draw(c, s));
  HIPCHK_C(hipStreamSynchronize(s));
  HIPCHK_C(hipGetLastError());
#undef ALLOC
#undef CHK
#undef HIPCHK_C
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(c);
  }
  *out = c;
  return IVHD_OK;
}

int ivhd_set_graphs(ivhd_ctx *ctx, int32_t enable) {
  if (!live(ctx)) return fail(IVHD_ESTATE, "invalid context");
  ctx->use_graphs = enable ? 1 : 0;
  return IVHD_OK;
}

int ivhd_step(ivhd_ctx *c, int64_t n_iters) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (n_iters < 0) return fail(IVHD_EINVAL, "n_iters = %lld < 0", (long long)n_iters);
  const int64_t R = c->p.rn > 0 ? c->p.rn_resample_every : 0;
  int64_t left = n_iters;
  int rc;
  while (left > 0) {
    if (R > 0) {
      const int64_t pos = c->n % R;
      const bool draw = (pos == 0 && c->n > 0);
      const int64_t chunk = left < R - pos ? left : R - pos;
      if (c->use_graphs && pos == 0 && chunk == R) {
        hipGraphExec_t &g = draw ? c->g_epoch[c->parity] : c->g_first[c->parity];
        if (!g && (rc = capture(c, draw, R, c->parity, &g))) return rc;
        HIPCHK(hipGraphLaunch(g, c->stream));
        if (c->det()) c->parity ^= (int)(R & 1);
      } else {
        if (draw && (rc = enqueue_draw(c, c->stream))) return rc;
        if ((rc = enqueue_steps(c, c->stream, chunk, &c->parity))) return rc;
      }
      c->n += chunk;
      left -= chunk;
    } else {
      if (c->use_graphs && left >= kChunkIters) {
        hipGraphExec_t &g = c->g_chunk[c->parity];
        if (!g && (rc = capture(c, false, kChunkIters, c->parity, &g))) return rc;
        HIPCHK(hipGraphLaunch(g, c->stream));
        c->n += kChunkIters;
        left -= kChunkIters;   // kChunkIters is even: parity unchanged
      } else {
        if ((rc = enqueue_steps(c, c->stream, left, &c->parity))) return rc;
        c->n += left;
        left = 0;
      }
    }
  }
  if (c->det() && c->parity) {
    HIPCHK(hipMemcpyAsync(c->y_user, c->y_alt, (size_t)c->p.M * sizeof(float2),
                          hipMemcpyDeviceToDevice, c->stream));
    c->parity = 0;
  }
  return IVHD_OK;
}

int ivhd_stress(ivhd_ctx *c, const float *d_y, double *h_E) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!h_E) return fail(IVHD_EINVAL, "h_E is NULL");
  const float2 *y = d_y ? (const float2 *)d_y : c->cur();
  HIPCHK(launch_stress(y, c->p.M, c->nn_idx, c->p.nn, c->rn_idx, c->p.rn, (double)c->p.c,
                       c->partials, c->nparts, c->d_E, c->stream));
  double E = 0.0;
  int32_t hflags[FLAG_SLOTS];
  HIPCHK(hipMemcpyAsync(&E, c->d_E, sizeof E, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(hflags, c->flags, sizeof hflags, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *h_E = E;
  if (hflags[FLAG_NONFINITE]) return fail(IVHD_ENUMERIC, "a non-finite position was produced by ivhd_step");
  if (!std::isfinite(E)) return fail(IVHD_ENUMERIC, "stress is not finite");
  return IVHD_OK;
}

int ivhd_grad(ivhd_ctx *c, const float *d_y, float *d_grad) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!d_grad) return fail(IVHD_EINVAL, "d_grad is NULL");
  const float2 *y = d_y ? (const float2 *)d_y : c->cur();
  StepArgs a = step_args(c, y, nullptr);
  if (c->det())
    HIPCHK(launch_grad_det(a, (float2 *)d_grad, c->stream));
  else
    HIPCHK(launch_grad_atomic(a, (float2 *)d_grad, c->stream));
  return IVHD_OK;
}

int ivhd_get_rn(ivhd_ctx *c, int32_t *d_rn_out) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (c->p.rn == 0) return IVHD_OK;
  if (!d_rn_out) return fail(IVHD_EINVAL, "d_rn_out is NULL");
  HIPCHK(hipMemcpyAsync(d_rn_out, c->rn_idx, (size_t)c->p.M * c->p.rn * sizeof(int32_t),
                        hipMemcpyDeviceToDevice, c->stream));
  return IVHD_OK;
}

int ivhd_get_in_edges(ivhd_ctx *c, int32_t which, int32_t *d_ptr, int32_t *d_src) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (which != 0 && which != 1) return fail(IVHD_EINVAL, "which = %d is neither 0 (nn) nor 1 (rn)", which);
  if (!d_ptr || !d_src) return fail(IVHD_EINVAL, "d_ptr or d_src is NULL");
  const Csc &g = which ? c->rn_csc : c->nn_csc;
  if (which == 1 && c->p.rn == 0) return IVHD_OK;
  if (which == 1 && !c->det()) return fail(IVHD_EINVAL, "atomic mode keeps no rn in-edge lists");
  const int64_t M = c->p.M;
  int32_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, g.ptr + M, sizeof total, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpyAsync(d_ptr, g.ptr, (size_t)(M + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  if (total > 0)
    HIPCHK(hipMemcpyAsync(d_src, g.src, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  return IVHD_OK;
}

int ivhd_get_iteration(const ivhd_ctx *c, int64_t *h_n) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!h_n) return fail(IVHD_EINVAL, "h_n is NULL");
  *h_n = c->n;
  return IVHD_OK;
}

// ---- edge plans: the stress and its gradient for caller-given edge lists ----

struct ivhd_edges {
  int64_t M = 0;
  int32_t nn = 0, rn = 0;
  const int32_t *nn_idx = nullptr, *rn_idx = nullptr;
  hipStream_t stream = nullptr;
  Csc nn_csc, rn_csc;
  CscScratch sc;
  int32_t *heavy = nullptr;
  int32_t n_heavy = 0;
  int32_t *flags = nullptr;
  double *partials = nullptr;
  int nparts = 0;
};

namespace {
std::mutex g_edges_mu;
std::unordered_set<const ivhd_edges *> g_edges_live;

bool edges_live(const ivhd_edges *e) {
  if (!e) return false;
  std::lock_guard<std::mutex> lk(g_edges_mu);
  return g_edges_live.count(e) != 0;
}

void free_edges(ivhd_edges *e) {
  if (!e) return;
  void *bufs[] = {e->nn_csc.ptr, e->nn_csc.src, e->rn_csc.ptr, e->rn_csc.src, e->sc.cnt,
                  e->sc.tmp, e->sc.part, e->sc.big, e->heavy, e->flags, e->partials};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete e;
}

StepArgs edge_args(const ivhd_edges *e, const float2 *y, float c, float eps, const float *gscale) {
  StepArgs a{};
  a.y = y;
  a.nn_idx = e->nn_idx;
  a.rn_idx = e->rn_idx;
  a.nn_ptr = e->nn_csc.ptr;
  a.nn_src = e->nn_csc.src;
  a.rn_ptr = e->rn_csc.ptr;
  a.rn_src = e->rn_csc.src;
  a.flags = e->flags;
  a.gscale = gscale;
  a.heavy = e->heavy;
  a.n_heavy = e->n_heavy;
  a.heavy_blocks = (e->n_heavy + kHeavyPerBlock - 1) / kHeavyPerBlock;
  a.M = e->M;
  a.nn = e->nn;
  a.rn = e->rn;
  a.c = c;
  a.eps = eps;
  return a;
}
}  // namespace

int ivhd_edges_create(ivhd_edges **out, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                      const int32_t *d_rn_idx, int32_t rn, void *stream) {
  clear_error();
  if (!out) return fail(IVHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (nn < 1 || nn > 64) return fail(IVHD_EINVAL, "nn = %d outside [1, 64]", nn);
  if (rn < 0 || rn > 64) return fail(IVHD_EINVAL, "rn = %d outside [0, 64]", rn);
  if (M * (int64_t)(nn > rn ? nn : rn) > (int64_t)INT32_MAX)
    return fail(IVHD_EINVAL, "M * max(nn, rn) exceeds 2^31-1 edges");
  if (!d_nn_idx) return fail(IVHD_EINVAL, "d_nn_idx is NULL");
  if (rn > 0 && !d_rn_idx) return fail(IVHD_EINVAL, "d_rn_idx is NULL while rn > 0");
  ivhd_edges *e = new (std::nothrow) ivhd_edges();
  if (!e) return fail(IVHD_ENOMEM, "host allocation of the edge plan failed");
  e->M = M;
  e->nn = nn;
  e->rn = rn;
  e->nn_idx = d_nn_idx;
  e->rn_idx = rn > 0 ? d_rn_idx : nullptr;
  e->stream = (hipStream_t)stream;
  const int64_t nb = (M + kScanChunk - 1) / kScanChunk;
  int rc;
#define E_CHK(expr)  \
  do {               \
    rc = (expr);     \
    if (rc) {        \
      free_edges(e); \
      return rc;     \
    }                \
  } while (0)
#define E_HIP(expr)                     \
  do {                                  \
    hipError_t _e = (expr);             \
    if (_e != hipSuccess) {             \
      rc = hip_fail(_e, #expr);         \
      free_edges(e);                    \
      return rc;                        \
    }                                   \
  } while (0)
  E_CHK(dev_alloc(&e->nn_csc.ptr, M + 1, "nn in-edge offsets"));
  E_CHK(dev_alloc(&e->nn_csc.src, M * nn, "nn in-edge sources"));
  if (rn > 0) {
    E_CHK(dev_alloc(&e->rn_csc.ptr, M + 1, "rn in-edge offsets"));
    E_CHK(dev_alloc(&e->rn_csc.src, M * rn, "rn in-edge sources"));
  }
  E_CHK(dev_alloc(&e->sc.cnt, M + 1, "CSC counts"));
  E_CHK(dev_alloc(&e->sc.tmp, M * (nn > rn ? nn : rn), "CSC scatter buffer"));
  E_CHK(dev_alloc(&e->sc.part, nb + 1, "scan partials"));
  E_CHK(dev_alloc(&e->sc.big, M, "large-segment list"));
  E_CHK(dev_alloc(&e->heavy, M, "heavy-vertex list"));
  E_CHK(dev_alloc(&e->flags, FLAG_SLOTS, "device flags"));
  e->nparts = stress_partials(M);
  E_CHK(dev_alloc(&e->partials, e->nparts, "stress partials"));
  hipStream_t s = e->stream;
  E_HIP(launch_fill_i32(e->flags, FLAG_SLOTS, 0, s));
  E_HIP(launch_validate_idx(d_nn_idx, M, nn, -1, e->flags, s));
  if (rn > 0) E_HIP(launch_validate_idx(d_rn_idx, M, rn, -1, e->flags, s));
  int32_t hflags[FLAG_SLOTS];
  E_HIP(hipMemcpyAsync(hflags, e->flags, sizeof hflags, hipMemcpyDeviceToHost, s));
  E_HIP(hipStreamSynchronize(s));
  if (hflags[FLAG_BAD_INDEX]) {
    free_edges(e);
    return fail(IVHD_EINVAL, "an nn or rn entry is outside [-1, M) or equals its row");
  }
  E_CHK(build_csc(d_nn_idx, M, nn, e->nn_csc, e->sc, e->flags, s));
  if (rn > 0) E_CHK(build_csc(d_rn_idx, M, rn, e->rn_csc, e->sc, e->flags, s));
  E_CHK(build_heavy(e->nn_csc, M, e->heavy, e->flags, &e->n_heavy, s));
#undef E_CHK
#undef E_HIP
  {
    std::lock_guard<std::mutex> lk(g_edges_mu);
    g_edges_live.insert(e);
  }
  *out = e;
  return IVHD_OK;
}

int ivhd_edges_stress(ivhd_edges *e, const float *d_y, float c, double *d_E) {
  if (!edges_live(e)) return fail(IVHD_ESTATE, "invalid edge plan");
  if (!d_y || !d_E) return fail(IVHD_EINVAL, "d_y and d_E must not be NULL");
  if (!std::isfinite(c) || c < 0.f) return fail(IVHD_EINVAL, "c = %g must be finite and >= 0", (double)c);
  HIPCHK(launch_stress((const float2 *)d_y, e->M, e->nn_idx, e->nn, e->rn_idx, e->rn, (double)c,
                       e->partials, e->nparts, d_E, e->stream));
  return IVHD_OK;
}

int ivhd_edges_grad(ivhd_edges *e, const float *d_y, float c, float eps, const float *d_scale,
                    float *d_grad) {
  if (!edges_live(e)) return fail(IVHD_ESTATE, "invalid edge plan");
  if (!d_y || !d_grad) return fail(IVHD_EINVAL, "d_y and d_grad must not be NULL");
  if (d_y == d_grad) return fail(IVHD_EINVAL, "d_y and d_grad alias");
  if (!std::isfinite(c) || c < 0.f) return fail(IVHD_EINVAL, "c = %g must be finite and >= 0", (double)c);
  if (!std::isfinite(eps) || eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)eps);
  HIPCHK(launch_grad_det(edge_args(e, (const float2 *)d_y, c, eps, d_scale), (float2 *)d_grad, e->stream));
  return IVHD_OK;
}

int ivhd_edges_destroy(ivhd_edges *e) {
  if (!e) return IVHD_OK;
  {
    std::lock_guard<std::mutex> lk(g_edges_mu);
    if (!g_edges_live.erase(e)) return fail(IVHD_ESTATE, "invalid edge plan");
  }
  hipError_t err = hipStreamSynchronize(e->stream);
  free_edges(e);
  if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
  return IVHD_OK;
}

int ivhd_grad_edges(const float *d_y, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                    const int32_t *d_rn_idx, int32_t rn, float c, float eps, float *d_grad,
                    double *h_E, void *stream) {
  ivhd_edges *e = nullptr;
  int rc = ivhd_edges_create(&e, M, d_nn_idx, nn, d_rn_idx, rn, stream);
  if (rc) return rc;
  rc = ivhd_edges_grad(e, d_y, c, eps, nullptr, d_grad);
  if (!rc && h_E) {
    double *d_E = nullptr;
    rc = dev_alloc(&d_E, 1, "stress result");
    if (!rc) rc = ivhd_edges_stress(e, d_y, c, d_E);
    if (!rc) {
      hipError_t err = hipMemcpyAsync(h_E, d_E, sizeof(double), hipMemcpyDeviceToHost, e->stream);
      if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
      if (err != hipSuccess) rc = hip_fail(err, "stress copy");
    }
    if (d_E) (void)hipFree(d_E);
  }
  int rc2 = ivhd_edges_destroy(e);
  return rc ? rc : rc2;
}

static int knn_common(const float *d_x, int64_t M, int32_t N, const float *d_q, int64_t Q,
                      int self_mode, const int32_t *d_self, int32_t k, int32_t *d_idx,
                      float *d_dist, void *stream) {
  if (!d_x || !d_q || !d_idx) return fail(IVHD_EINVAL, "d_x, d_q and d_idx must not be NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (N < 1) return fail(IVHD_EINVAL, "N = %d must be >= 1", N);
  if (Q < 0) return fail(IVHD_EINVAL, "Q = %lld < 0", (long long)Q);
  const int64_t kmax = M - 1 < knn_max_k() ? M - 1 : knn_max_k();
  if (k < 1 || k > kmax) return fail(IVHD_EINVAL, "k = %d outside [1, %lld]", k, (long long)kmax);
  if (Q == 0) return IVHD_OK;
  hipStream_t s = (hipStream_t)stream;
  float *norms = nullptr;
  int rc = dev_alloc(&norms, (size_t)M, "row norms");
  if (rc) return rc;
  hipError_t e = launch_row_norms(d_x, M, N, norms, s);
  if (e == hipSuccess) e = launch_knn(d_x, M, N, d_q, Q, self_mode, d_self, norms, k, d_idx, d_dist, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(norms);
  if (e != hipSuccess) return hip_fail(e, "knn");
  return IVHD_OK;
}

int ivhd_knn_build(const float *d_x, int64_t M, int32_t N, int32_t k, int32_t *d_idx, void *stream) {
  return knn_common(d_x, M, N, d_x, M, 1, nullptr, k, d_idx, nullptr, stream);
}

int ivhd_knn_query(const float *d_x, int64_t M, int32_t N, const float *d_q, int64_t Q,
                   const int32_t *d_self, int32_t k, int32_t *d_idx, float *d_dist, void *stream) {
  return knn_common(d_x, M, N, d_q, Q, d_self ? 2 : 0, d_self, k, d_idx, d_dist, stream);
}

int ivhd_destroy(ivhd_ctx *c) {
  if (!c) return IVHD_OK;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!g_live.erase(c)) return fail(IVHD_ESTATE, "invalid context");
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  free_ctx(c);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return IVHD_OK;
}

}  // extern "C"
