// The internal vertex order of a context built with IVHD_FLAG_REORDER.
//
// Vertices are grouped by connected component of the undirected nn graph
// (components ordered by their smallest id), inside a component by nn
// in-degree, capped at the hub threshold + 1, then by their first nn
// neighbour (absent last), then by id.
//
// Why: the deterministic step gives one thread to each light vertex, and a
// wavefront lasts as long as its slowest lane.  kNN graphs of
// high-dimensional data are hubby: in a random order most wavefronts hold a
// vertex of in-degree 15 or more while the mean is 2, so most lanes idle
// through chains of dependent gathers.  Sorting by in-degree makes the lanes
// of a wavefront walk lists of nearly equal length.  Grouping by component
// keeps every nn gather of a tile inside one component's stretch of Y, which
// the XCD-aware tile mapping of the step kernel then keeps in one L2.
// Among vertices of equal in-degree (most have none), those pointing at the
// same hub sit side by side: a wavefront's out-edge gathers then hit the same
// positions, and a hub's in-edge sources form runs of consecutive ids.
//
// The order is two stable LSD radix sorts over the ids 0..M-1: first by the
// first neighbour, then by (root << 7) | capped degree; a pure function of
// the nn lists.
#include <hipcub/hipcub.hpp>

#include "ivhd_internal.h"

namespace ivhd {
namespace {

constexpr int kDegreeBits = 7;
static_assert(kHeavyDegree + 1 < (1 << kDegreeBits), "degree cap must fit the key's low bits");

__global__ void first_neighbour_keys_kernel(const int32_t *__restrict__ nn_idx, int nn, int64_t M,
                                            uint32_t *__restrict__ keys, int32_t *__restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int32_t j = nn_idx[i * nn];
  keys[i] = j >= 0 ? (uint32_t)j : 0xffffffffu;
  ids[i] = (int32_t)i;
}

// the component / degree key of the vertices in the order of the first pass
__global__ void order_keys_kernel(const int32_t *__restrict__ root, const int32_t *__restrict__ indeg,
                                  const int32_t *__restrict__ ids, int64_t M, int cap,
                                  uint64_t *__restrict__ keys) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= M) return;
  const int32_t i = ids[p];
  const int32_t d = indeg[i] < cap ? indeg[i] : cap;
  keys[p] = ((uint64_t)(uint32_t)root[i] << kDegreeBits) | (uint64_t)d;
}

}  // namespace

int sort_vertex_order(const int32_t *root, const int32_t *indeg, const int32_t *nn_idx, int nn, int64_t M,
                      int heavy_deg, int32_t *perm, hipStream_t s) {
  if (heavy_deg < 0 || heavy_deg + 1 >= (1 << kDegreeBits)) return fail(IVHD_EINVAL, "hub threshold %d", heavy_deg);
  int end_bit = kDegreeBits;
  while ((int64_t{1} << (end_bit - kDegreeBits)) < M) ++end_bit;
  uint32_t *k1 = nullptr, *k1_out = nullptr;
  uint64_t *k2 = nullptr, *k2_out = nullptr;
  int32_t *ids = nullptr, *ids1 = nullptr;
  void *temp = nullptr;
  size_t t1 = 0, t2 = 0;
  int rc = IVHD_OK;
  auto cleanup = [&]() {
    void *bufs[] = {k1, k1_out, k2, k2_out, ids, ids1, temp};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
  };
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, t1, k1, k1_out, ids, ids1, (int)M, 0, 32, s);
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, t2, k2, k2_out, ids1, perm, (int)M, 0, end_bit, s);
  if (e != hipSuccess) return hip_fail(e, "radix sort size query");
  const size_t temp_bytes = t1 > t2 ? t1 : t2;
  if ((rc = dev_alloc(&k1, M, "first-neighbour keys")) || (rc = dev_alloc(&k1_out, M, "sorted first-neighbour keys")) ||
      (rc = dev_alloc(&k2, M, "order keys")) || (rc = dev_alloc(&k2_out, M, "sorted order keys")) ||
      (rc = dev_alloc(&ids, M, "vertex ids")) || (rc = dev_alloc(&ids1, M, "vertex ids by first neighbour")) ||
      (rc = dev_alloc((uint8_t **)&temp, temp_bytes, "sort scratch"))) {
    cleanup();
    return rc;
  }
  size_t tb = temp_bytes;
  first_neighbour_keys_kernel<<<grid_for(M), kBlock, 0, s>>>(nn_idx, nn, M, k1, ids);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortPairs(temp, tb, k1, k1_out, ids, ids1, (int)M, 0, 32, s);
  if (e == hipSuccess) {
    order_keys_kernel<<<grid_for(M), kBlock, 0, s>>>(root, indeg, ids1, M, heavy_deg + 1, k2);
    e = hipGetLastError();
  }
  tb = temp_bytes;
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(temp, tb, k2, k2_out, ids1, perm, (int)M, 0, end_bit, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // before the scratch is freed
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "sorting the vertex order");
  return IVHD_OK;
}

int build_vertex_order(const int32_t *nn_idx, int64_t M, int nn, int heavy_deg, int32_t *parent, int32_t *indeg,
                       int32_t *changed, int32_t *perm, int32_t *inv, hipStream_t s) {
  HIPCHK(launch_cc_init(parent, M, s));
  for (int rounds = 0;; ++rounds) {
    if (rounds >= kCcMaxRounds) return fail(IVHD_EDEVICE, "connected components did not converge");
    int32_t h = 0;
    HIPCHK(launch_fill_i32(changed, 1, 0, s));
    HIPCHK(launch_cc_round(nn_idx, M, nn, parent, changed, s));
    HIPCHK(hipMemcpyAsync(&h, changed, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!h) break;
  }
  HIPCHK(launch_fill_i32(indeg, M + 1, 0, s));
  HIPCHK(launch_count(nn_idx, M, nn, indeg, s));
  const int rc = sort_vertex_order(parent, indeg, nn_idx, nn, M, heavy_deg, perm, s);
  if (rc) return rc;
  HIPCHK(launch_inverse_perm(perm, M, inv, s));
  return IVHD_OK;
}

}  // namespace ivhd
