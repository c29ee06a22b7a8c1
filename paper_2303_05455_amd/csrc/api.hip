// Host side of the loop part of the C ABI (include/ivhd.h): argument
// validation, context lifetime, the internal vertex order, the random-
// neighbour epochs, the ping-pong of the positions and the HIP-graph replay
// of the iteration loop.
//
// The context keeps the embedding in its own buffers, in an internal vertex
// order: with IVHD_FLAG_REORDER the vertices are grouped by connected
// component of the nn graph (every nn edge then joins vertices of one
// contiguous block of ids, and the XCD-aware tiles of the step kernel keep
// those blocks in one L2).  The caller's buffers receive the state, in the
// caller's order, at the end of every ivhd_step.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>

#include "ivhd_internal.h"

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
  return fail(e == hipErrorOutOfMemory ? IVHD_ENOMEM : IVHD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

}  // namespace ivhd

using namespace ivhd;

namespace {

// contexts handed out and not yet destroyed: a stale or foreign pointer is
// reported as IVHD_ESTATE instead of being dereferenced
std::mutex g_live_mu;
std::unordered_set<const ivhd_ctx *> g_live;

constexpr int kChunkIters = 64;   // graph length when random neighbours are drawn once

}  // namespace

struct ivhd_ctx {
  ivhd_params p{};
  hipStream_t stream = nullptr;   // caller's
  hipStream_t cap = nullptr;      // private stream used only for graph capture
  const int32_t *nn_user = nullptr;   // caller's nn lists (caller ids)
  float2 *y_user = nullptr, *v_user = nullptr;
  int32_t *perm = nullptr;        // internal p -> caller id (NULL: identity)
  int32_t *inv = nullptr;         // caller id -> internal p
  int32_t *nn_own = nullptr;      // nn lists in internal ids (when reordered)
  const int32_t *nn_int = nullptr;   // the lists the kernels read
  float2 *ya = nullptr, *yb = nullptr, *v = nullptr;   // internal state
  float2 *ha = nullptr, *hb = nullptr;   // Nesterov look-ahead H = Y + a V (det: paired with ya / yb)
  float2 *vb = nullptr;                  // adaptive b: second velocity buffer (paired with v)
  AdaptState *adapt = nullptr;           // adaptive b: device state
  double *ke_part = nullptr;             // adaptive b: per-block kinetic energy changes
  int adapt_on = 0;
  double tau = 0.0;
  float g1 = 1.f, g2 = 1.f;
  float2 *s2 = nullptr;                  // Adam: second moments (v holds the first)
  AdamState *adam = nullptr;             // Adam: step count and bias corrections
  int adam_on = 0;
  float lr = 0.f, beta1 = 0.9f, beta2 = 0.999f, eps_adam = 1e-8f;
  float2 *tmp = nullptr;          // [M] scratch (gradients in internal order)
  int parity = 0;                 // det mode: 0 -> Y_n in ya, 1 -> in yb
  Csc nn_csc, rn_csc;
  CscScratch sc;
  int32_t *rn_idx = nullptr;      // internal ids, internal row order
  int64_t *epoch = nullptr;
  int32_t *flags = nullptr;
  float2 *fbuf = nullptr;
  float2 *fown = nullptr;
  uint64_t *facc = nullptr;       // atomic mode: fixed-point rn reactions
  ReactionRange *rx = nullptr;    // atomic mode: their range for the current draw
  int32_t *fflag = nullptr;       // atomic mode: [2] float-accumulator flags
  int32_t fpar = 0;               // atomic mode: flag slot of the next iteration
  int32_t *heavy = nullptr;
  int32_t n_heavy = 0;
  int32_t heavy_deg = kHeavyDegree;
  double *partials = nullptr;
  int nparts = 0;
  double *d_E = nullptr;
  int64_t n = 0;
  int use_graphs = 1;
  hipGraphExec_t g_epoch[2] = {nullptr, nullptr};   // draw + R iterations
  hipGraphExec_t g_first[2] = {nullptr, nullptr};   // the R iterations of epoch 0
  hipGraphExec_t g_chunk[2] = {nullptr, nullptr};   // kChunkIters iterations (no draws)

  bool det() const { return p.mode == IVHD_MODE_DET; }
  bool nest() const { return (p.flags & IVHD_FLAG_NESTEROV) != 0; }
  bool l1() const { return (p.flags & IVHD_FLAG_L1) != 0; }
  float2 *cur() const { return parity ? yb : ya; }
  float2 *other() const { return parity ? ya : yb; }
  float2 *vcur() const { return adapt_on && parity ? vb : v; }
  float2 *hcur() const { return det() && parity ? hb : ha; }
};

namespace {

void free_ctx(ivhd_ctx *c) {
  if (!c) return;
  for (int k = 0; k < 2; ++k) {
    if (c->g_epoch[k]) (void)hipGraphExecDestroy(c->g_epoch[k]);
    if (c->g_first[k]) (void)hipGraphExecDestroy(c->g_first[k]);
    if (c->g_chunk[k]) (void)hipGraphExecDestroy(c->g_chunk[k]);
  }
  void *bufs[] = {c->perm, c->inv, c->nn_own, c->ya, c->yb, c->v, c->tmp, c->nn_csc.ptr, c->nn_csc.src,
                  c->rn_csc.ptr, c->rn_csc.src, c->sc.cnt, c->sc.tmp, c->sc.part, c->sc.big, c->sc.rank, c->rn_idx,
                  c->epoch, c->flags, c->fbuf, c->fown, c->facc, c->rx, c->fflag, c->heavy, c->partials, c->d_E, c->ha, c->hb, c->vb,
                  c->adapt, c->ke_part, c->s2, c->adam};
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
    return fail(IVHD_EINVAL, "nn + rn = %d exceeds M - 1 = %lld", p->nn + p->rn, (long long)(p->M - 1));
  if (p->M * (int64_t)(p->nn > p->rn ? p->nn : p->rn) > (int64_t)INT32_MAX)
    return fail(IVHD_EINVAL, "M * max(nn, rn) exceeds 2^31-1 edges");
  if (!std::isfinite(p->a) || p->a < 0.f || p->a > 1.f) return fail(IVHD_EINVAL, "a = %g outside [0, 1]", (double)p->a);
  if (!std::isfinite(p->b) || !(p->b > 0.f)) return fail(IVHD_EINVAL, "b = %g must be > 0", (double)p->b);
  if (!std::isfinite(p->c) || !(p->c > 0.f) || !(p->c < 1.f))
    return fail(IVHD_EINVAL, "c = %g outside (0, 1)", (double)p->c);
  if (!std::isfinite(p->eps) || p->eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)p->eps);
  if (p->rn_resample_every < 0)
    return fail(IVHD_EINVAL, "rn_resample_every = %d must be >= 0", p->rn_resample_every);
  if (p->mode != IVHD_MODE_DET && p->mode != IVHD_MODE_ATOMIC)
    return fail(IVHD_EINVAL, "mode = %d is neither IVHD_MODE_DET nor IVHD_MODE_ATOMIC", p->mode);
  if (p->flags & ~(IVHD_FLAG_REORDER | IVHD_FLAG_NESTEROV | IVHD_FLAG_L1))
    return fail(IVHD_EINVAL, "flags = 0x%x has unknown bits", (unsigned)p->flags);
  if (p->reserved != 0) return fail(IVHD_EINVAL, "reserved = %d must be 0", p->reserved);
  return IVHD_OK;
}

StepArgs step_args(const ivhd_ctx *c, const float2 *y, float2 *y_out) {
  StepArgs a{};
  a.y = y;
  a.h = y;
  a.y_out = y_out;
  a.v = c->v;
  a.l1 = c->l1() ? 1 : 0;
  a.nn_idx = c->nn_int;
  a.rn_idx = c->rn_idx;
  a.nn_ptr = c->nn_csc.ptr;
  a.nn_src = c->nn_csc.src;
  a.rn_ptr = c->rn_csc.ptr;
  a.rn_src = c->rn_csc.src;
  a.fbuf = c->fbuf;
  a.fown = c->fown;
  a.facc = c->facc;
  a.rx = c->rx;
  a.fflag = c->fflag;
  a.rx_unit = ldexpf(c->p.c, -kReactionFracBits);
  a.rx_inv_unit = ldexpf(1.f / c->p.c, kReactionFracBits);
  a.flags = c->flags;
  a.gscale = nullptr;
  a.heavy = c->heavy;
  a.n_heavy = c->n_heavy;
  a.heavy_deg = c->heavy_deg;
  a.M = c->p.M;
  a.nn = c->p.nn;
  a.rn = c->p.rn;
  a.a = c->p.a;
  a.b = c->p.b;
  a.c = c->p.c;
  a.eps = c->p.eps;
  set_launch_shape(a);
  return a;
}

// A new random-neighbour epoch: epoch += 1, draw, count the rn in-degrees,
// then rebuild the transposed rn lists (det mode) or set the fixed-point
// range of the rn reactions (atomic mode).
int enqueue_draw(ivhd_ctx *c, hipStream_t s) {
  if (c->p.rn == 0) return IVHD_OK;
  const int64_t M = c->p.M;
  int32_t *cnt = c->sc.cnt;
  HIPCHK(launch_epoch_begin(c->epoch, cnt, M, c->flags, s));
  HIPCHK(launch_rn_sample(c->nn_user, M, c->p.nn, c->p.rn, c->p.seed, c->epoch, c->perm, c->inv, c->rn_idx, cnt,
                          c->det() ? c->sc.rank : nullptr, s));
  if (c->det()) {
    HIPCHK(launch_scan(c->sc.cnt, M, c->sc.part, c->rn_csc.ptr, s));
    HIPCHK(launch_place_sort(c->rn_idx, M, c->p.rn, c->rn_csc.ptr, c->sc.rank, c->sc.tmp, c->sc.big, c->flags,
                             c->rn_csc.src, s));
  } else {
    HIPCHK(launch_reaction_range(cnt, M, c->rx, s));
  }
  return IVHD_OK;
}

// `count` iterations starting from parity *par.  Det mode ping-pongs Y (and
// H for Nesterov, V for the adaptive b) between the two buffers of a pair;
// after a rejected adaptive step the commit kernel copies the state across,
// so the pairing stays static (and capturable).
int enqueue_steps(ivhd_ctx *c, hipStream_t s, int64_t count, int *par) {
  for (int64_t k = 0; k < count; ++k) {
    if (c->det()) {
      float2 *src = *par ? c->yb : c->ya;
      float2 *dst = *par ? c->ya : c->yb;
      StepArgs a = step_args(c, src, dst);
      if (c->nest()) {
        a.opt = OPT_NEST;
        a.h = *par ? c->hb : c->ha;
        a.h_out = *par ? c->ha : c->hb;
      }
      if (c->adam_on) {
        a.opt = OPT_ADAM;
        a.s2 = c->s2;
        a.adam = c->adam;
        a.lr = c->lr;
        a.beta1 = c->beta1;
        a.beta2 = c->beta2;
        a.eps_adam = c->eps_adam;
        HIPCHK(launch_adam_prep(c->adam, c->beta1, c->beta2, s));
      }
      if (c->adapt_on) {
        a.opt = OPT_ADAPT;
        a.v = *par ? c->vb : c->v;
        a.v_out = *par ? c->v : c->vb;
        a.b_dev = &c->adapt->b;
        a.ke_part = c->ke_part;
      }
      HIPCHK(launch_step_det(a, s));
      if (c->adapt_on) {
        HIPCHK(launch_adapt_decide(c->ke_part, (int)det_grid(a), c->tau, c->g1, c->g2, c->adapt, s));
        HIPCHK(launch_adapt_commit(c->adapt, src, a.v, c->p.M, dst, a.v_out, s));
      }
      *par ^= 1;
    } else {
      StepArgs a = step_args(c, c->ya, c->ya);
      a.fpar = c->fpar;
      c->fpar ^= 1;
      if (c->nest()) {
        a.opt = OPT_NEST;
        a.h = c->ha;
        a.h_out = c->ha;
      }
      HIPCHK(launch_step_atomic(a, s));
    }
  }
  return IVHD_OK;
}

void drop_graphs(ivhd_ctx *c) {
  for (int k = 0; k < 2; ++k) {
    hipGraphExec_t *gs[] = {&c->g_epoch[k], &c->g_first[k], &c->g_chunk[k]};
    for (hipGraphExec_t *g : gs)
      if (*g) {
        (void)hipGraphExecDestroy(*g);
        *g = nullptr;
      }
  }
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

// the internal order: vertices grouped by connected component of the nn
// graph (components by their smallest caller id), inside a component by nn
// in-degree capped at the hub threshold + 1, then by first nn neighbour,
// then by caller id
int build_order(ivhd_ctx *c) {
  const int64_t M = c->p.M;
  hipStream_t s = c->stream;
  // parent: nn_own ([M*nn] >= M ints) is free until the lists are mapped;
  // indeg: the CSC counts are free until the nn lists are transposed
  int rc = build_vertex_order(c->nn_user, M, c->p.nn, c->heavy_deg, c->nn_own, c->sc.cnt, c->flags + 3, c->perm,
                              c->inv, s);
  if (rc) return rc;
  HIPCHK(launch_map_lists(c->nn_user, M, c->p.nn, c->perm, c->inv, c->nn_own, s));
  return IVHD_OK;
}

// caller state -> internal state (order and buffers)
int load_state(ivhd_ctx *c, const float2 *y, const float2 *v) {
  HIPCHK(launch_gather_f2(y, c->perm, c->p.M, c->ya, c->stream));
  HIPCHK(launch_gather_f2(v, c->perm, c->p.M, c->v, c->stream));
  c->parity = 0;
  if (c->nest()) HIPCHK(launch_lookahead(c->ya, c->v, c->p.a, c->p.M, c->ha, c->stream));
  return IVHD_OK;
}

// internal state -> caller's buffers
int store_state(ivhd_ctx *c) {
  HIPCHK(launch_gather_f2(c->cur(), c->inv, c->p.M, c->y_user, c->stream));
  HIPCHK(launch_gather_f2(c->vcur(), c->inv, c->p.M, c->v_user, c->stream));
  return IVHD_OK;
}

// d_y in the caller's order -> internal order in the spare position buffer
const float2 *internal_positions(ivhd_ctx *c, const float *d_y, int *rc) {
  *rc = IVHD_OK;
  if (!d_y) return c->cur();
  hipError_t e = launch_gather_f2((const float2 *)d_y, c->perm, c->p.M, c->other(), c->stream);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "gather of the given positions");
    return nullptr;
  }
  return c->other();
}

}  // namespace

extern "C" {

const char *ivhd_last_error(void) { return ivhd::g_err.c_str(); }

int ivhd_version(void) { return 300; }

int ivhd_init(ivhd_ctx **out, const ivhd_params *p, const int32_t *d_nn_idx, float *d_y, float *d_v,
              void *stream) {
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
  c->nn_user = d_nn_idx;
  c->y_user = (float2 *)d_y;
  c->v_user = (float2 *)d_v;
  const int64_t M = p->M;
  const int64_t nb = (M + kScanChunk - 1) / kScanChunk;
  const int64_t cap_tmp = M * (int64_t)(p->nn > p->rn ? p->nn : p->rn);
  const bool reorder = (p->flags & IVHD_FLAG_REORDER) != 0;

#define ALLOC(ptr, n, what)                    \
  do {                                         \
    rc = dev_alloc(&(ptr), (size_t)(n), what); \
    if (rc) {                                  \
      free_ctx(c);                             \
      return rc;                               \
    }                                          \
  } while (0)
#define CHK(expr)  \
  do {             \
    rc = (expr);   \
    if (rc) {      \
      free_ctx(c); \
      return rc;   \
    }              \
  } while (0)
#define HIPCHK_C(expr)          \
  do {                          \
    hipError_t _e = (expr);     \
    if (_e != hipSuccess) {     \
      rc = hip_fail(_e, #expr); \
      free_ctx(c);              \
      return rc;                \
    }                           \
  } while (0)

  HIPCHK_C(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  ALLOC(c->ya, M, "positions");
  ALLOC(c->yb, M, "second position buffer");
  ALLOC(c->v, M, "velocities");
  ALLOC(c->tmp, M, "gradient scratch");
  ALLOC(c->nn_csc.ptr, M + 1, "nn in-edge offsets");
  ALLOC(c->nn_csc.src, M * p->nn, "nn in-edge sources");
  ALLOC(c->sc.cnt, M + 1, "CSC counts");
  ALLOC(c->sc.tmp, cap_tmp, "CSC scatter buffer");
  ALLOC(c->sc.part, nb + 1, "scan partials");
  ALLOC(c->sc.big, M, "large-segment list");
  ALLOC(c->epoch, 1, "epoch counter");
  ALLOC(c->flags, FLAG_SLOTS, "device flags");
  if (reorder) {
    ALLOC(c->perm, M, "vertex order");
    ALLOC(c->inv, M, "inverse vertex order");
    ALLOC(c->nn_own, M * p->nn, "nn lists in internal order");
  }
  if (p->rn > 0) {
    ALLOC(c->rn_idx, M * p->rn, "random neighbours");
    if (p->mode == IVHD_MODE_DET) {
      ALLOC(c->rn_csc.ptr, M + 1, "rn in-edge offsets");
      ALLOC(c->rn_csc.src, M * p->rn, "rn in-edge sources");
      ALLOC(c->sc.rank, M * p->rn, "rn arrival ranks");
    }
  }
  if (p->mode == IVHD_MODE_ATOMIC) {
    ALLOC(c->fbuf, M, "rn reaction accumulator (float)");
    ALLOC(c->fown, M, "own force shares");
    ALLOC(c->facc, M, "rn reaction accumulator (fixed point)");
    ALLOC(c->rx, 1, "fixed-point range of the rn reactions");
    ALLOC(c->fflag, 2, "float reaction flags");
  }
  if (p->flags & IVHD_FLAG_NESTEROV) {
    ALLOC(c->ha, M, "look-ahead positions");
    if (p->mode == IVHD_MODE_DET) ALLOC(c->hb, M, "second look-ahead buffer");
  }
  ALLOC(c->heavy, M, "heavy-vertex list");
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
  c->heavy_deg = heavy_degree(M);
  if (reorder) {
    CHK(build_order(c));
    c->nn_int = c->nn_own;
  } else {
    c->nn_int = d_nn_idx;
  }
  CHK(build_csc(c->nn_int, M, p->nn, c->nn_csc, c->sc, c->flags, s));
  if (c->heavy) CHK(build_heavy(c->nn_csc, M, c->heavy_deg, c->heavy, c->flags, &c->n_heavy, s));
  if (c->fbuf) HIPCHK_C(launch_fill_i32((int32_t *)c->fbuf, 2 * M, 0, s));
  if (c->facc) HIPCHK_C(launch_fill_i32((int32_t *)c->facc, 2 * M, 0, s));
  if (c->fflag) HIPCHK_C(launch_fill_i32(c->fflag, 2, 0, s));
  CHK(load_state(c, c->y_user, c->v_user));
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
  return n_iters > 0 ? store_state(c) : IVHD_OK;
}

int ivhd_set_state(ivhd_ctx *c, const float *d_y, const float *d_v) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!d_y || !d_v) return fail(IVHD_EINVAL, "d_y and d_v must not be NULL");
  return load_state(c, (const float2 *)d_y, (const float2 *)d_v);
}

int ivhd_set_iteration(ivhd_ctx *c, int64_t n) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (n < 0) return fail(IVHD_EINVAL, "n = %lld < 0", (long long)n);
  const int64_t R = c->p.rn > 0 ? c->p.rn_resample_every : 0;
  // the draw held before iteration n: epoch (n - 1) / R (epoch 0 at n = 0)
  const int64_t e = (R > 0 && n > 0) ? (n - 1) / R : 0;
  if (c->p.rn > 0) {
    const int64_t before = e - 1;
    HIPCHK(hipMemcpyAsync(c->epoch, &before, sizeof before, hipMemcpyHostToDevice, c->stream));
    int rc = enqueue_draw(c, c->stream);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));   // `before` lives on this stack frame
  }
  c->n = n;
  return IVHD_OK;
}

int ivhd_stress(ivhd_ctx *c, const float *d_y, double *h_E) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!h_E) return fail(IVHD_EINVAL, "h_E is NULL");
  int rc;
  const float2 *y = internal_positions(c, d_y, &rc);
  if (rc) return rc;
  HIPCHK(launch_stress(y, c->p.M, c->nn_int, c->p.nn, c->rn_idx, c->p.rn, (double)c->p.c, c->l1() ? 1 : 0,
                       c->partials,
                       c->nparts, c->d_E, c->stream));
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
  int rc;
  const float2 *y = internal_positions(c, d_y, &rc);
  if (rc) return rc;
  StepArgs a = step_args(c, y, nullptr);
  if (c->det()) {
    HIPCHK(launch_grad_det(a, c->tmp, c->stream));
  } else {
    a.fpar = c->fpar;
    c->fpar ^= 1;
    HIPCHK(launch_grad_atomic(a, c->tmp, c->stream));
  }
  HIPCHK(launch_gather_f2(c->tmp, c->inv, c->p.M, (float2 *)d_grad, c->stream));
  return IVHD_OK;
}

int ivhd_get_rn(ivhd_ctx *c, int32_t *d_rn_out) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (c->p.rn == 0) return IVHD_OK;
  if (!d_rn_out) return fail(IVHD_EINVAL, "d_rn_out is NULL");
  if (c->perm) {
    HIPCHK(launch_unmap_lists(c->rn_idx, c->p.M, c->p.rn, c->perm, c->inv, d_rn_out, c->stream));
  } else {
    HIPCHK(hipMemcpyAsync(d_rn_out, c->rn_idx, (size_t)c->p.M * c->p.rn * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, c->stream));
  }
  return IVHD_OK;
}

int ivhd_get_order(ivhd_ctx *c, int32_t *d_perm) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!d_perm) return fail(IVHD_EINVAL, "d_perm is NULL");
  if (c->perm) {
    HIPCHK(hipMemcpyAsync(d_perm, c->perm, (size_t)c->p.M * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(launch_cc_init(d_perm, c->p.M, c->stream));   // identity
  }
  return IVHD_OK;
}

int ivhd_get_in_edges(ivhd_ctx *c, int32_t which, int32_t *d_ptr, int32_t *d_src) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (which != 0 && which != 1) return fail(IVHD_EINVAL, "which = %d is neither 0 (nn) nor 1 (rn)", which);
  if (!d_ptr || !d_src) return fail(IVHD_EINVAL, "d_ptr or d_src is NULL");
  if (which == 1 && c->p.rn == 0) return IVHD_OK;
  if (which == 1 && !c->det()) return fail(IVHD_EINVAL, "atomic mode keeps no rn in-edge lists");
  const Csc &g = which ? c->rn_csc : c->nn_csc;
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

int ivhd_set_adaptive(ivhd_ctx *c, int32_t enable, float b, double tau, float g1, float g2) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!enable) {
    if (c->adapt_on) {
      if (c->parity) HIPCHK(hipMemcpyAsync(c->v, c->vb, (size_t)c->p.M * sizeof(float2), hipMemcpyDeviceToDevice,
                                           c->stream));
      c->adapt_on = 0;
      drop_graphs(c);
    }
    return IVHD_OK;
  }
  if (!c->det()) return fail(IVHD_EINVAL, "the adaptive b needs IVHD_MODE_DET");
  if (c->nest()) return fail(IVHD_EINVAL, "the adaptive b is not combined with IVHD_FLAG_NESTEROV");
  if (c->adam_on) return fail(IVHD_EINVAL, "the adaptive b is not combined with Adam");
  if (!std::isfinite(b) || !(b > 0.f)) return fail(IVHD_EINVAL, "b = %g must be > 0", (double)b);
  if (std::isnan(tau) || tau < 0.0) return fail(IVHD_EINVAL, "tau = %g must be >= 0", tau);
  if (!std::isfinite(g1) || !(g1 > 1.f)) return fail(IVHD_EINVAL, "g1 = %g must be > 1", (double)g1);
  if (!std::isfinite(g2) || !(g2 > 0.f) || !(g2 < 1.f)) return fail(IVHD_EINVAL, "g2 = %g outside (0, 1)", (double)g2);
  const int64_t M = c->p.M;
  int rc;
  if (!c->vb && (rc = dev_alloc(&c->vb, M, "second velocity buffer"))) return rc;
  if (!c->adapt && (rc = dev_alloc(&c->adapt, 1, "adaptive-b state"))) return rc;
  if (!c->ke_part) {
    const StepArgs a = step_args(c, c->ya, c->yb);
    if ((rc = dev_alloc(&c->ke_part, det_grid(a), "kinetic energy partials"))) return rc;
  }
  if (!c->adapt_on && c->parity)
    HIPCHK(hipMemcpyAsync(c->vb, c->v, (size_t)M * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
  AdaptState st{};
  st.b = b;
  HIPCHK(hipMemcpyAsync(c->adapt, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));   // st lives on this stack frame
  c->adapt_on = 1;
  c->tau = tau;
  c->g1 = g1;
  c->g2 = g2;
  drop_graphs(c);
  return IVHD_OK;
}

int ivhd_set_adam(ivhd_ctx *c, int32_t enable, float lr, float beta1, float beta2, float eps) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!enable) {
    if (c->adam_on) {
      c->adam_on = 0;
      drop_graphs(c);
    }
    return IVHD_OK;
  }
  if (!c->det()) return fail(IVHD_EINVAL, "Adam needs IVHD_MODE_DET");
  if (c->nest()) return fail(IVHD_EINVAL, "Adam is not combined with IVHD_FLAG_NESTEROV");
  if (c->adapt_on) return fail(IVHD_EINVAL, "Adam is not combined with the adaptive b");
  if (!std::isfinite(lr) || !(lr > 0.f)) return fail(IVHD_EINVAL, "lr = %g must be > 0", (double)lr);
  if (!std::isfinite(beta1) || beta1 < 0.f || !(beta1 < 1.f))
    return fail(IVHD_EINVAL, "beta1 = %g outside [0, 1)", (double)beta1);
  if (!std::isfinite(beta2) || beta2 < 0.f || !(beta2 < 1.f))
    return fail(IVHD_EINVAL, "beta2 = %g outside [0, 1)", (double)beta2);
  if (!std::isfinite(eps) || !(eps > 0.f)) return fail(IVHD_EINVAL, "eps = %g must be > 0", (double)eps);
  const int64_t M = c->p.M;
  int rc;
  if (!c->s2 && (rc = dev_alloc(&c->s2, M, "second moments"))) return rc;
  if (!c->adam && (rc = dev_alloc(&c->adam, 1, "Adam state"))) return rc;
  // fresh moments: V (the first moments) and the second moments start at zero
  HIPCHK(launch_fill_i32((int32_t *)c->v, 2 * M, 0, c->stream));
  HIPCHK(launch_fill_i32((int32_t *)c->s2, 2 * M, 0, c->stream));
  AdamState st{};
  HIPCHK(hipMemcpyAsync(c->adam, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));   // st lives on this stack frame
  c->adam_on = 1;
  c->lr = lr;
  c->beta1 = beta1;
  c->beta2 = beta2;
  c->eps_adam = eps;
  drop_graphs(c);
  return IVHD_OK;
}

int ivhd_get_adaptive(ivhd_ctx *c, float *h_b, int64_t *h_kept, int64_t *h_rejected, double *h_dT) {
  if (!live(c)) return fail(IVHD_ESTATE, "invalid context");
  if (!c->adapt) return fail(IVHD_EINVAL, "the adaptive b was never enabled on this context");
  AdaptState st{};
  HIPCHK(hipMemcpyAsync(&st, c->adapt, sizeof st, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h_b) *h_b = st.b;
  if (h_kept) *h_kept = st.kept;
  if (h_rejected) *h_rejected = st.rejected;
  if (h_dT) *h_dT = st.dT;
  return IVHD_OK;
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
