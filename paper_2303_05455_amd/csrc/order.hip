// The internal vertex order of a context built with IVHD_FLAG_REORDER.
//
// Vertices are grouped by connected component of the undirected nn graph
// (components ordered by their smallest id), and inside a component by nn
// in-degree, capped at the hub threshold + 1, ties by id.
//
// Why: the deterministic step gives one thread to each light vertex, and a
// wavefront lasts as long as its slowest lane.  kNN graphs of
// high-dimensional data are hubby: in a random order most wavefronts hold a
// vertex of in-degree 15 or more while the mean is 2, so most lanes idle
// through chains of dependent gathers.  Sorting by in-degree makes the lanes
// of a wavefront walk lists of nearly equal length.  Grouping by component
// keeps every nn gather of a tile inside one component's stretch of Y, which
// the XCD-aware tile mapping of the step kernel then keeps in one L2.
//
// The order is a stable LSD radix sort of the key (root << 7) | capped degree
// over the ids 0..M-1, so it is a pure function of the nn lists.
#include <hipcub/hipcub.hpp>

#include "ivhd_internal.h"

namespace ivhd {
namespace {

constexpr int kDegreeBits = 7;
static_assert(kHeavyDegree + 1 < (1 << kDegreeBits), "degree cap must fit the key's low bits");

__global__ void order_keys_kernel(const int32_t *__restrict__ root, const int32_t *__restrict__ indeg,
                                  int64_t M, int cap, uint64_t *__restrict__ keys, int32_t *__restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int32_t d = indeg[i] < cap ? indeg[i] : cap;
  keys[i] = ((uint64_t)(uint32_t)root[i] << kDegreeBits) | (uint64_t)d;
  ids[i] = (int32_t)i;
}

}  // namespace

int sort_vertex_order(const int32_t *root, const int32_t *indeg, int64_t M, int heavy_deg, int32_t *perm,
                      hipStream_t s) {
  if (heavy_deg < 0 || heavy_deg + 1 >= (1 << kDegreeBits)) return fail(IVHD_EINVAL, "hub threshold %d", heavy_deg);
  int end_bit = kDegreeBits;
  while ((int64_t{1} << (end_bit - kDegreeBits)) < M) ++end_bit;
  uint64_t *keys = nullptr, *keys_out = nullptr;
  int32_t *ids = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int rc = IVHD_OK;
  auto cleanup = [&]() {
    void *bufs[] = {keys, keys_out, ids, temp};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
  };
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys, keys_out, ids, perm, (int)M, 0,
                                                    end_bit, s);
  if (e != hipSuccess) return hip_fail(e, "radix sort size query");
  if ((rc = dev_alloc(&keys, M, "order keys")) || (rc = dev_alloc(&keys_out, M, "sorted order keys")) ||
      (rc = dev_alloc(&ids, M, "vertex ids")) || (rc = dev_alloc((uint8_t **)&temp, temp_bytes, "sort scratch"))) {
    cleanup();
    return rc;
  }
  order_keys_kernel<<<grid_for(M), kBlock, 0, s>>>(root, indeg, M, heavy_deg + 1, keys, ids);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_out, ids, perm, (int)M, 0, end_bit, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // before the scratch is freed
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "sorting the vertex order");
  return IVHD_OK;
}

}  // namespace ivhd
