// Host side of the stateless parts of the C ABI: edge plans (the stress and
// its gradient for caller-given edge lists) and the exact kNN builder.
#include <cmath>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include <cstring>

#include "ivhd_internal.h"

using namespace ivhd;

namespace ivhd {

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

// measured: 70,000 vertices (nn = 5) 9.6 us per step at 16 against 11.2 us at
// 80; 1.4M vertices (nn = 2) 67.9 us at 80 against 69.2 at 48 and 69.0 at 100
int heavy_degree(int64_t M) { return M < kSmallGraphVertices ? kSmallGraphHeavyDegree : kHeavyDegree; }

// the vertices of nn in-degree above heavy_deg; synchronises s to read the count
int build_heavy(const Csc &nn_csc, int64_t M, int heavy_deg, int32_t *heavy, int32_t *flags, int32_t *n_heavy,
                hipStream_t s) {
  HIPCHK(launch_fill_i32(flags + FLAG_BIG_COUNT, 1, 0, s));
  HIPCHK(launch_heavy_list(nn_csc.ptr, M, heavy_deg, heavy, flags + FLAG_BIG_COUNT, s));
  HIPCHK(hipMemcpyAsync(n_heavy, flags + FLAG_BIG_COUNT, sizeof *n_heavy, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return IVHD_OK;
}

}  // namespace ivhd

extern "C" {

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
  int32_t heavy_deg = kHeavyDegree;
  int32_t *flags = nullptr;
  double *partials = nullptr;
  int nparts = 0;
  // IVHD_EDGES_REORDER: internal vertex order (NULL: the caller's)
  int32_t *perm = nullptr, *inv = nullptr;   // internal p -> caller id, and back
  int32_t *nn_own = nullptr, *rn_own = nullptr;   // the lists in internal ids and order
  float2 *yp = nullptr;                      // the layout gathered into the internal order
  double *gparts = nullptr;                  // per-block stress of the fused gradient kernel
  int ngparts = 0;
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
  void *bufs[] = {e->nn_csc.ptr, e->nn_csc.src, e->rn_csc.ptr, e->rn_csc.src, e->sc.cnt, e->sc.tmp,
                  e->sc.part, e->sc.big, e->heavy, e->flags, e->partials, e->perm, e->inv,
                  e->nn_own, e->rn_own, e->yp, e->gparts};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete e;
}

StepArgs edge_args(const ivhd_edges *e, const float2 *y, float c, float eps, const float *gscale) {
  StepArgs a{};
  a.y = y;
  a.h = y;
  a.nn_idx = e->nn_idx;
  a.rn_idx = e->rn_idx;
  a.nn_ptr = e->nn_csc.ptr;
  a.nn_src = e->nn_csc.src;
  a.rn_ptr = e->rn_csc.ptr;
  a.rn_src = e->rn_csc.src;
  a.flags = e->flags;
  a.gscale = gscale;
  a.out_perm = e->perm;
  a.heavy = e->heavy;
  a.n_heavy = e->n_heavy;
  a.heavy_deg = e->heavy_deg;
  a.M = e->M;
  a.nn = e->nn;
  a.rn = e->rn;
  a.c = c;
  a.eps = eps;
  set_launch_shape(a);
  return a;
}
}  // namespace

int ivhd_edges_create(ivhd_edges **out, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                      const int32_t *d_rn_idx, int32_t rn, int32_t flags, void *stream) {
  clear_error();
  if (!out) return fail(IVHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (flags & ~IVHD_EDGES_REORDER) return fail(IVHD_EINVAL, "unknown flags 0x%x", (unsigned)flags);
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
  e->heavy_deg = heavy_degree(M);
  if (flags & IVHD_EDGES_REORDER) {
    E_CHK(dev_alloc(&e->perm, M, "vertex order"));
    E_CHK(dev_alloc(&e->inv, M, "inverse vertex order"));
    E_CHK(dev_alloc(&e->nn_own, M * nn, "nn lists in internal order"));
    if (rn > 0) E_CHK(dev_alloc(&e->rn_own, M * rn, "rn lists in internal order"));
    E_CHK(dev_alloc(&e->yp, M, "layout in internal order"));
    // nn_own ([M*nn] >= M ints) is the component scratch until the lists are mapped
    E_CHK(build_vertex_order(d_nn_idx, M, nn, e->heavy_deg, e->nn_own, e->sc.cnt, e->flags + 3, e->perm, e->inv,
                             s));
    E_HIP(launch_map_lists(d_nn_idx, M, nn, e->perm, e->inv, e->nn_own, s));
    if (rn > 0) E_HIP(launch_map_lists(d_rn_idx, M, rn, e->perm, e->inv, e->rn_own, s));
    e->nn_idx = e->nn_own;
    e->rn_idx = e->rn_own;
  }
  E_CHK(build_csc(e->nn_idx, M, nn, e->nn_csc, e->sc, e->flags, s));
  if (rn > 0) E_CHK(build_csc(e->rn_idx, M, rn, e->rn_csc, e->sc, e->flags, s));
  E_CHK(build_heavy(e->nn_csc, M, e->heavy_deg, e->heavy, e->flags, &e->n_heavy, s));
  e->ngparts = (int)det_grid(edge_args(e, nullptr, 0.f, 0.f, nullptr));
  E_CHK(dev_alloc(&e->gparts, e->ngparts, "fused stress partials"));
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
  const float2 *y = (const float2 *)d_y;
  if (e->perm) {
    HIPCHK(launch_gather_f2(y, e->perm, e->M, e->yp, e->stream));
    y = e->yp;
  }
  HIPCHK(launch_stress(y, e->M, e->nn_idx, e->nn, e->rn_idx, e->rn, (double)c, 0, e->partials, e->nparts, d_E,
                       e->stream));
  return IVHD_OK;
}

int ivhd_edges_grad(ivhd_edges *e, const float *d_y, float c, float eps, const float *d_scale,
                    float *d_grad) {
  if (!edges_live(e)) return fail(IVHD_ESTATE, "invalid edge plan");
  if (!d_y || !d_grad) return fail(IVHD_EINVAL, "d_y and d_grad must not be NULL");
  if (d_y == d_grad) return fail(IVHD_EINVAL, "d_y and d_grad alias");
  if (!std::isfinite(c) || c < 0.f) return fail(IVHD_EINVAL, "c = %g must be finite and >= 0", (double)c);
  if (!std::isfinite(eps) || eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)eps);
  const float2 *y = (const float2 *)d_y;
  if (e->perm) {
    HIPCHK(launch_gather_f2(y, e->perm, e->M, e->yp, e->stream));
    y = e->yp;
  }
  HIPCHK(launch_grad_det(edge_args(e, y, c, eps, d_scale), (float2 *)d_grad, e->stream));
  return IVHD_OK;
}

int ivhd_edges_stress_grad(ivhd_edges *e, const float *d_y, float c, float eps, const float *d_scale,
                           double *d_E, float *d_grad) {
  if (!edges_live(e)) return fail(IVHD_ESTATE, "invalid edge plan");
  if (!d_y || !d_E || !d_grad) return fail(IVHD_EINVAL, "d_y, d_E and d_grad must not be NULL");
  if (d_y == d_grad) return fail(IVHD_EINVAL, "d_y and d_grad alias");
  if (!std::isfinite(c) || c < 0.f) return fail(IVHD_EINVAL, "c = %g must be finite and >= 0", (double)c);
  if (!std::isfinite(eps) || eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)eps);
  const float2 *y = (const float2 *)d_y;
  if (e->perm) {
    HIPCHK(launch_gather_f2(y, e->perm, e->M, e->yp, e->stream));
    y = e->yp;
  }
  StepArgs a = edge_args(e, y, c, eps, d_scale);
  a.e_part = e->gparts;
  HIPCHK(launch_grad_det(a, (float2 *)d_grad, e->stream));
  HIPCHK(launch_stress_final(e->gparts, e->ngparts, d_E, e->stream));
  return IVHD_OK;
}

int ivhd_scale_f32(const float *d_x, int64_t n, const float *d_scale, float *d_out, void *stream) {
  if (n < 0) return fail(IVHD_EINVAL, "n = %lld < 0", (long long)n);
  if (n == 0) return IVHD_OK;
  if (!d_x || !d_scale || !d_out) return fail(IVHD_EINVAL, "d_x, d_scale and d_out must not be NULL");
  HIPCHK(launch_scale_f32(d_x, n, d_scale, d_out, (hipStream_t)stream));
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
  int rc = ivhd_edges_create(&e, M, d_nn_idx, nn, d_rn_idx, rn, 0, stream);
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
  const bool same = d_q == d_x && Q == M;
  const int Np = knn_padded_width(N);
  float *norms = nullptr;
  uint32_t *amax = nullptr;
  _Float16 *xs = nullptr, *qs = nullptr;   // [2][rows][Np]: hi then lo
  int rc = dev_alloc(&norms, (size_t)M, "row norms");
  if (!rc) rc = dev_alloc(&amax, 1, "largest magnitude");
  if (!rc) rc = dev_alloc(&xs, (size_t)2 * M * Np, "split rows of X");
  if (!rc && !same) rc = dev_alloc(&qs, (size_t)2 * Q * Np, "split rows of the queries");
  auto cleanup = [&]() {
    void *bufs[] = {norms, amax, xs, qs};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
  };
  if (rc) {
    cleanup();
    return rc;
  }
  uint32_t bits = 0;
  hipError_t e = hipMemsetAsync(amax, 0, sizeof *amax, s);
  if (e == hipSuccess) e = launch_absmax(d_x, M * (int64_t)N, amax, s);
  if (e == hipSuccess && !same) e = launch_absmax(d_q, Q * (int64_t)N, amax, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&bits, amax, sizeof bits, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "knn input scan");
  }
  float amx;
  std::memcpy(&amx, &bits, sizeof amx);
  if (!std::isfinite(amx)) {
    cleanup();
    return fail(IVHD_EINVAL, "the points hold a non-finite coordinate");
  }
  const float scale = knn_split_scale(amx);
  _Float16 *qh = same ? xs : qs, *ql = same ? xs + M * Np : qs + Q * Np;
  e = launch_row_norms(d_x, M, N, norms, s);
  if (e == hipSuccess) e = launch_split(d_x, M, N, Np, scale, xs, xs + M * Np, s);
  if (e == hipSuccess && !same) e = launch_split(d_q, Q, N, Np, scale, qs, qs + Q * Np, s);
  if (e == hipSuccess)
    e = launch_knn(d_x, M, N, d_q, Q, xs, xs + M * Np, qh, ql, Np, scale, self_mode, d_self, norms, k, d_idx, d_dist,
                   s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
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

}  // extern "C"

namespace ivhd {
namespace {

// device buffers released together
struct Scratch {
  std::vector<void *> bufs;
  ~Scratch() {
    for (void *b : bufs)
      if (b) (void)hipFree(b);
  }
  template <typename T>
  int get(T **p, size_t n, const char *what) {
    int rc = dev_alloc(p, n, what);
    if (!rc) bufs.push_back(*p);
    return rc;
  }
};

// per-target lists of a rows x k index array (targets in [0, ntargets)):
// ptr [ntargets+1], src [rows*k]
int transpose_lists(Scratch &S, const int32_t *idx, int64_t rows, int k, int64_t ntargets, int32_t **ptr,
                    int32_t **src, int32_t *flags, hipStream_t s) {
  int32_t *cnt, *part, *tmp, *big;
  int rc;
  if ((rc = S.get(ptr, ntargets + 1, "list offsets")) || (rc = S.get(src, rows * k, "list members")) ||
      (rc = S.get(&cnt, ntargets + 1, "list counts")) ||
      (rc = S.get(&part, ntargets / kScanChunk + 2, "scan partials")) ||
      (rc = S.get(&tmp, rows * k, "scatter buffer")) || (rc = S.get(&big, ntargets, "large-list list")))
    return rc;
  HIPCHK(launch_transpose(idx, rows, k, ntargets, *ptr, cnt, part, tmp, big, flags, *src, s));
  return IVHD_OK;
}

int check_range(const int32_t *idx, int64_t n, int32_t hi, int32_t *flags, hipStream_t s, const char *what) {
  int32_t h[FLAG_SLOTS] = {0};
  HIPCHK(launch_fill_i32(flags, FLAG_SLOTS, 0, s));
  HIPCHK(launch_range_check(idx, n, hi, flags, s));
  HIPCHK(hipMemcpyAsync(h, flags, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h[FLAG_BAD_INDEX]) return fail(IVHD_EINVAL, "%s holds an entry outside [0, %d)", what, hi);
  return IVHD_OK;
}

}  // namespace
}  // namespace ivhd

extern "C" {

int ivhd_ivf_train(const float *d_x, int64_t M, int32_t N, int32_t nlist, int32_t n_iter, float *d_centroids,
                   int32_t *d_assign, void *stream) {
  clear_error();
  if (!d_x || !d_centroids || !d_assign) return fail(IVHD_EINVAL, "d_x, d_centroids and d_assign must not be NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (N < 1) return fail(IVHD_EINVAL, "N = %d must be >= 1", N);
  if (nlist < 2 || nlist > M) return fail(IVHD_EINVAL, "nlist = %d outside [2, M]", nlist);
  if (n_iter < 0) return fail(IVHD_EINVAL, "n_iter = %d < 0", n_iter);
  hipStream_t s = (hipStream_t)stream;
  Scratch S;
  int32_t *flags;
  int rc = S.get(&flags, FLAG_SLOTS, "device flags");
  if (rc) return rc;
  HIPCHK(launch_init_centroids(d_x, M, N, nlist, d_centroids, s));
  for (int it = 0; it <= n_iter; ++it) {
    if ((rc = ivhd_knn_query(d_centroids, nlist, N, d_x, M, nullptr, 1, d_assign, nullptr, stream))) return rc;
    if (it == n_iter) break;
    Scratch L;
    int32_t *lptr, *pos_id;
    if ((rc = transpose_lists(L, d_assign, M, 1, nlist, &lptr, &pos_id, flags, s))) return rc;
    HIPCHK(launch_centroid_mean(d_x, N, lptr, pos_id, nlist, d_centroids, s));
    HIPCHK(hipStreamSynchronize(s));   // before L frees the lists
  }
  return IVHD_OK;
}

int ivhd_ivf_search(const float *d_x, int64_t M, int32_t N, const float *d_centroids, int32_t nlist,
                    const int32_t *d_assign, const float *d_q, int64_t Q, const int32_t *d_self, int32_t k,
                    int32_t nprobe, int32_t *d_idx, float *d_dist, void *stream) {
  clear_error();
  if (!d_x || !d_centroids || !d_assign || !d_q || !d_idx) return fail(IVHD_EINVAL, "a required pointer is NULL");
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (N < 1) return fail(IVHD_EINVAL, "N = %d must be >= 1", N);
  if (nlist < 2 || nlist > M) return fail(IVHD_EINVAL, "nlist = %d outside [2, M]", nlist);
  if (Q < 0 || Q > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "Q = %lld outside [0, 2^31-2]", (long long)Q);
  const int32_t kmax = knn_max_k() < M - 1 ? knn_max_k() : (int32_t)(M - 1);
  if (k < 1 || k > kmax) return fail(IVHD_EINVAL, "k = %d outside [1, %d]", k, kmax);
  const int32_t pmax = knn_max_k() < nlist - 1 ? knn_max_k() : nlist - 1;
  if (nprobe < 1 || nprobe > pmax) return fail(IVHD_EINVAL, "nprobe = %d outside [1, %d]", nprobe, pmax);
  if (Q * (int64_t)nprobe > (int64_t)INT32_MAX) return fail(IVHD_EINVAL, "Q * nprobe exceeds 2^31-1");
  if (Q == 0) return IVHD_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch S;
  int32_t *flags;
  int rc = S.get(&flags, FLAG_SLOTS, "device flags");
  if (rc) return rc;
  if ((rc = check_range(d_assign, M, nlist, flags, s, "d_assign"))) return rc;
  // probes: the nprobe nearest centroids of every query
  int32_t *probes;
  if ((rc = S.get(&probes, Q * nprobe, "probes"))) return rc;
  if ((rc = ivhd_knn_query(d_centroids, nlist, N, d_q, Q, nullptr, nprobe, probes, nullptr, stream))) return rc;
  // lists (points by list, ids ascending) and, per list, its probing queries
  int32_t *lptr, *pos_id, *pptr, *pq;
  if ((rc = transpose_lists(S, d_assign, M, 1, nlist, &lptr, &pos_id, flags, s))) return rc;
  if ((rc = transpose_lists(S, probes, Q, nprobe, nlist, &pptr, &pq, flags, s))) return rc;
  // work items: (list, chunk of 128 probing queries)
  std::vector<int32_t> hp(nlist + 1), wl, wc;
  HIPCHK(hipMemcpyAsync(hp.data(), pptr, (nlist + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t c = 0; c < nlist; ++c)
    for (int32_t h = 0; (int64_t)h * 128 < (int64_t)hp[c + 1] - hp[c]; ++h) {
      wl.push_back(c);
      wc.push_back(h);
    }
  const int64_t n_work = (int64_t)wl.size();
  int32_t *d_wl, *d_wc;
  if ((rc = S.get(&d_wl, n_work, "work lists")) || (rc = S.get(&d_wc, n_work, "work chunks"))) return rc;
  if (n_work) {
    HIPCHK(hipMemcpyAsync(d_wl, wl.data(), n_work * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_wc, wc.data(), n_work * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  // split rows at one scale: points in list order, queries in their own order
  uint32_t *amax;
  if ((rc = S.get(&amax, 1, "largest magnitude"))) return rc;
  uint32_t bits = 0;
  HIPCHK(hipMemsetAsync(amax, 0, sizeof *amax, s));
  HIPCHK(launch_absmax(d_x, M * (int64_t)N, amax, s));
  HIPCHK(launch_absmax(d_q, Q * (int64_t)N, amax, s));
  HIPCHK(hipMemcpyAsync(&bits, amax, sizeof bits, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));   // also orders the host vectors' copies above
  float amx;
  std::memcpy(&amx, &bits, sizeof amx);
  if (!std::isfinite(amx)) return fail(IVHD_EINVAL, "the points hold a non-finite coordinate");
  const float scale = knn_split_scale(amx);
  const int Np = knn_padded_width(N);
  _Float16 *xs, *qs;
  float *norms, *pnorm, *part_dist;
  int32_t *part_idx;
  if ((rc = S.get(&xs, (size_t)2 * M * Np, "split points")) || (rc = S.get(&qs, (size_t)2 * Q * Np, "split queries")) ||
      (rc = S.get(&norms, M, "row norms")) || (rc = S.get(&pnorm, M, "row norms in list order")) ||
      (rc = S.get(&part_idx, Q * nprobe * k, "per-probe results")) ||
      (rc = S.get(&part_dist, Q * nprobe * k, "per-probe distances")))
    return rc;
  HIPCHK(launch_split_gather(d_x, M, N, Np, scale, pos_id, xs, xs + M * Np, s));
  HIPCHK(launch_split(d_q, Q, N, Np, scale, qs, qs + Q * Np, s));
  HIPCHK(launch_row_norms(d_x, M, N, norms, s));
  HIPCHK(launch_gather_f32(norms, pos_id, M, pnorm, s));
  HIPCHK(launch_fill_i32(part_idx, Q * nprobe * k, -1, s));
  HIPCHK(launch_ivf_lists(d_x, N, d_q, xs, xs + M * Np, qs, qs + Q * Np, Np, scale, pnorm, pos_id, lptr, pptr, pq,
                          d_wl, d_wc, n_work, probes, nprobe, d_self, k, part_idx, part_dist, s));
  HIPCHK(launch_ivf_merge(part_idx, part_dist, Q, nprobe, k, d_idx, d_dist, s));
  HIPCHK(hipStreamSynchronize(s));
  return IVHD_OK;
}

int ivhd_rnn_mask(const int32_t *d_nn_idx, int64_t M, int32_t nn, const int32_t *d_helper, int32_t kh,
                  int32_t *d_out, void *stream) {
  clear_error();
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (nn < 1 || nn > 64) return fail(IVHD_EINVAL, "nn = %d outside [1, 64]", nn);
  if (kh < 1 || kh > 256) return fail(IVHD_EINVAL, "kh = %d outside [1, 256]", kh);
  if (M * (int64_t)(nn > kh ? nn : kh) > (int64_t)INT32_MAX)
    return fail(IVHD_EINVAL, "M * max(nn, kh) exceeds 2^31-1");
  if (!d_nn_idx || !d_helper || !d_out) return fail(IVHD_EINVAL, "a list pointer is NULL");
  if (d_helper == d_out) return fail(IVHD_EINVAL, "d_helper and d_out alias");
  hipStream_t s = (hipStream_t)stream;
  int32_t *flags = nullptr;
  int rc = dev_alloc(&flags, FLAG_SLOTS, "device flags");
  if (rc) return rc;
  int32_t hflags[FLAG_SLOTS] = {0};
  hipError_t e = launch_fill_i32(flags, FLAG_SLOTS, 0, s);
  if (e == hipSuccess) e = launch_validate_idx(d_nn_idx, M, nn, -1, flags, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flags);
  if (e != hipSuccess) return hip_fail(e, "validating nn_idx");
  if (hflags[FLAG_BAD_INDEX]) return fail(IVHD_EINVAL, "nn_idx holds an entry outside [-1, M) or a self edge");
  HIPCHK(launch_rnn_mask(d_nn_idx, M, nn, d_helper, kh, d_out, s));
  return IVHD_OK;
}

}  // extern "C"

#include "ivhd_probe.h"

extern "C" int ivhd_probe_gather(const float *d_src, int64_t n_src, const int32_t *d_idx, int64_t n, float *d_dst,
                                 void *stream) {
  clear_error();
  if (n < 0 || n_src < 1) return fail(IVHD_EINVAL, "n = %lld and n_src = %lld must be >= 0 and >= 1",
                                      (long long)n, (long long)n_src);
  if (n == 0) return IVHD_OK;
  if (!d_src || !d_idx || !d_dst) return fail(IVHD_EINVAL, "d_src, d_idx and d_dst must not be NULL");
  HIPCHK(launch_gather_f2((const float2 *)d_src, d_idx, n, (float2 *)d_dst, (hipStream_t)stream));
  return IVHD_OK;
}

extern "C" int ivhd_probe_atomic(uint64_t *d_acc, int64_t n_acc, const int32_t *d_idx, int64_t n, void *stream) {
  clear_error();
  if (n < 0 || n_acc < 1) return fail(IVHD_EINVAL, "n = %lld and n_acc = %lld must be >= 0 and >= 1",
                                      (long long)n, (long long)n_acc);
  if (n == 0) return IVHD_OK;
  if (!d_acc || !d_idx) return fail(IVHD_EINVAL, "d_acc and d_idx must not be NULL");
  HIPCHK(launch_probe_atomic(d_acc, d_idx, n, (hipStream_t)stream));
  return IVHD_OK;
}
