// ivhd_grad_edges_noalloc: the one-shot stress gradient of ivhd_grad_edges
// for callers that cannot allocate device memory.
//
// Everything ivhd_grad_edges keeps in a temporary edge plan (the transposed
// nn and rn lists, the transpose scratch, the hub list, the device flags,
// the FP64 stress partials and the stress result) lives here in one
// file-scope device array instead.  Each GPU the library runs on holds its
// own copy of the array until the process ends; its device address is looked
// up once per device with hipGetSymbolAddress and only that address is
// handed to kernels and copies (the array's name is a host-side stand-in in
// host code).  The kernels are the ones ivhd_grad_edges launches, so the
// results are the same bit for bit.
//
// Every call on a GPU shares that GPU's array and leaves its contents
// behind; each call clears what must start at zero (the flags and the
// transpose counters) with fill kernels.  The call synchronises its stream
// before returning, so calls made one after another never overlap; calls
// that overlap on one GPU (other threads or streams) race on the array.
#include <cmath>
#include <mutex>

#include "ivhd_internal.h"

using namespace ivhd;

constexpr size_t kNoAllocScratchBytes = size_t{64} << 20;   // 64 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// carves consecutive 256-byte aligned pieces out of [base, base + bytes)
struct Carver {
  unsigned char *base;
  size_t used = 0;
  template <typename T>
  T *take(size_t count) {
    T *p = base ? (T *)(base + used) : nullptr;
    used += (count * sizeof(T) + kAlign - 1) / kAlign * kAlign;
    return p;
  }
};

struct NoAllocLayout {
  Csc nn_csc, rn_csc;
  CscScratch sc;
  int32_t *heavy, *flags;
  double *partials, *E;
  int nparts;
  size_t bytes;
};

// the pieces of one call; base = NULL only measures
NoAllocLayout carve(unsigned char *base, int64_t M, int32_t nn, int32_t rn) {
  NoAllocLayout L{};
  Carver c{base};
  const int64_t nb = (M + kScanChunk - 1) / kScanChunk;
  L.nn_csc.ptr = c.take<int32_t>(M + 1);
  L.nn_csc.src = c.take<int32_t>(M * nn);
  if (rn > 0) {
    L.rn_csc.ptr = c.take<int32_t>(M + 1);
    L.rn_csc.src = c.take<int32_t>(M * rn);
  }
  L.sc.cnt = c.take<int32_t>(M + 1);
  L.sc.tmp = c.take<int32_t>(M * (nn > rn ? nn : rn));
  L.sc.part = c.take<int32_t>(nb + 1);
  L.sc.big = c.take<int32_t>(M);
  L.heavy = c.take<int32_t>(M);
  L.flags = c.take<int32_t>(FLAG_SLOTS);
  L.nparts = stress_partials(M);
  L.partials = c.take<double>(L.nparts);
  L.E = c.take<double>(1);
  L.bytes = c.used;
  return L;
}

// device address of this device's scratch array (looked up once per device)
int scratch_address(unsigned char **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(IVHD_EDEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(IVHD_EDEVICE, "no device address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char *)g_scratch_ptr[dev];
  return IVHD_OK;
}

}  // namespace

extern "C" {

int ivhd_grad_edges_noalloc(const float *d_y, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                            const int32_t *d_rn_idx, int32_t rn, float c, float eps, float *d_grad,
                            double *h_E, void *stream) {
  clear_error();
  if (M < 2 || M > (int64_t)INT32_MAX - 1) return fail(IVHD_EINVAL, "M = %lld outside [2, 2^31-2]", (long long)M);
  if (nn < 1 || nn > 64) return fail(IVHD_EINVAL, "nn = %d outside [1, 64]", nn);
  if (rn < 0 || rn > 64) return fail(IVHD_EINVAL, "rn = %d outside [0, 64]", rn);
  if (M * (int64_t)(nn > rn ? nn : rn) > (int64_t)INT32_MAX)
    return fail(IVHD_EINVAL, "M * max(nn, rn) exceeds 2^31-1 edges");
  if (!d_nn_idx) return fail(IVHD_EINVAL, "d_nn_idx is NULL");
  if (rn > 0 && !d_rn_idx) return fail(IVHD_EINVAL, "d_rn_idx is NULL while rn > 0");
  if (!d_y || !d_grad) return fail(IVHD_EINVAL, "d_y and d_grad must not be NULL");
  if (d_y == d_grad) return fail(IVHD_EINVAL, "d_y and d_grad alias");
  if (!std::isfinite(c) || c < 0.f) return fail(IVHD_EINVAL, "c = %g must be finite and >= 0", (double)c);
  if (!std::isfinite(eps) || eps < 0.f) return fail(IVHD_EINVAL, "eps = %g must be >= 0", (double)eps);
  const size_t need = carve(nullptr, M, nn, rn).bytes;
  if (need > kNoAllocScratchBytes)
    return fail(IVHD_EINVAL, "M = %lld, nn = %d, rn = %d needs %zu bytes of scratch, above the %zu-byte limit",
                (long long)M, nn, rn, need, kNoAllocScratchBytes);

  unsigned char *base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  const NoAllocLayout L = carve(base, M, nn, rn);
  hipStream_t s = (hipStream_t)stream;

  HIPCHK(launch_fill_i32(L.flags, FLAG_SLOTS, 0, s));
  HIPCHK(launch_validate_idx(d_nn_idx, M, nn, -1, L.flags, s));
  if (rn > 0) HIPCHK(launch_validate_idx(d_rn_idx, M, rn, -1, L.flags, s));
  int32_t hflags[FLAG_SLOTS];
  HIPCHK(hipMemcpyAsync(hflags, L.flags, sizeof hflags, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hflags[FLAG_BAD_INDEX]) return fail(IVHD_EINVAL, "an nn or rn entry is outside [-1, M) or equals its row");

  Csc nn_csc = L.nn_csc, rn_csc = L.rn_csc;
  CscScratch sc = L.sc;
  if ((rc = build_csc(d_nn_idx, M, nn, nn_csc, sc, L.flags, s))) return rc;
  if (rn > 0 && (rc = build_csc(d_rn_idx, M, rn, rn_csc, sc, L.flags, s))) return rc;
  int32_t n_heavy = 0;
  const int heavy_deg = heavy_degree(M);
  if ((rc = build_heavy(nn_csc, M, heavy_deg, L.heavy, L.flags, &n_heavy, s))) return rc;

  StepArgs a{};
  a.y = (const float2 *)d_y;
  a.h = a.y;
  a.nn_idx = d_nn_idx;
  a.rn_idx = rn > 0 ? d_rn_idx : nullptr;
  a.nn_ptr = nn_csc.ptr;
  a.nn_src = nn_csc.src;
  a.rn_ptr = rn_csc.ptr;
  a.rn_src = rn_csc.src;
  a.flags = L.flags;
  a.gscale = nullptr;
  a.heavy = L.heavy;
  a.n_heavy = n_heavy;
  a.heavy_deg = heavy_deg;
  a.M = M;
  a.nn = nn;
  a.rn = rn;
  a.c = c;
  a.eps = eps;
  set_launch_shape(a);
  HIPCHK(launch_grad_det(a, (float2 *)d_grad, s));
  if (h_E) {
    HIPCHK(launch_stress(a.y, M, d_nn_idx, nn, a.rn_idx, rn, (double)c, 0, L.partials, L.nparts, L.E, s));
    HIPCHK(hipMemcpyAsync(h_E, L.E, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return IVHD_OK;
}

}  // extern "C"
