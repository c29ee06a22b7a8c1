// Graph structures of the IVHD loop on gfx950:
//  * validation of the caller's nn lists,
//  * the random-neighbour draw (rn random non-neighbours per vertex, drawn
//    ad hoc, never an nn neighbour: Sec. "Improving classical MDS" and the
//    practical rules of Sec. "Force directed"), keyed SplitMix64 counters,
//  * the transposed (in-edge) lists that let every vertex gather the
//    reactions of the edges pointing at it without atomics.  The IVHD-CUDA
//    section writes each connection's +/- force to two slots instead; here
//    each edge is recomputed at both ends, which moves fewer bytes.
//
// CSC build: in-degree count -> exclusive scan -> atomic-cursor scatter ->
// per-segment sort by source, so the final order is canonical (sources
// ascending) whatever order the atomics ran in.  Segments up to 32 entries
// are insertion-sorted by one thread; longer ones (kNN hubs) by one block
// each with a bitonic network whose comparators all point the same way,
// which lets a segment of any length be sorted in place (the virtual +inf
// padding never moves).
#include "ivhd_internal.h"

namespace ivhd {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void validate_idx_kernel(const int32_t *__restrict__ idx, int64_t M, int k, int32_t lo,
                                    int32_t *flags) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  int64_t i = e / k;
  int64_t j = idx[e];
  if (j < lo || j >= M || j == i) flags[FLAG_BAD_INDEX] = 1;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t value) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = value;
}

__global__ void epoch_begin_kernel(int64_t *epoch, int32_t *cnt, int64_t M, int32_t *flags) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) {
    *epoch = *epoch + 1;
    if (cnt) flags[FLAG_BIG_COUNT] = 0;
  }
  if (cnt && e <= M) cnt[e] = 0;
}

// perm / inv (both NULL or both set): the draw is defined on the caller's
// vertex ids; thread p serves internal vertex p = inv[i], i = perm[p], and
// stores the internal id inv[j] of each draw j
__global__ void rn_sample_kernel(const int32_t *__restrict__ nn_idx, int64_t M, int nn, int rn,
                                 uint64_t seed, const int64_t *__restrict__ epoch_p,
                                 const int32_t *__restrict__ perm, const int32_t *__restrict__ inv,
                                 int32_t *__restrict__ rn_idx, int32_t *__restrict__ cnt,
                                 int32_t *__restrict__ rank) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= M) return;
  const int64_t i = perm ? (int64_t)perm[p] : p;
  const uint64_t e = (uint64_t)(*epoch_p);
  const uint64_t range = (uint64_t)(M - 1);
  for (int r = 0; r < rn; ++r) {
    int32_t pick = -1;
    for (int t = 0; t < 256; ++t) {
      uint64_t ctr = ((e * (uint64_t)M + (uint64_t)i) * (uint64_t)rn + (uint64_t)r) * 256u + (uint64_t)t;
      uint64_t h = splitmix64(seed ^ splitmix64(ctr));
      int64_t j = (int64_t)(h % range);
      if (j >= i) j += 1;
      const int32_t js = inv ? inv[j] : (int32_t)j;
      bool clash = false;
      for (int q = 0; q < nn; ++q) clash |= (nn_idx[i * nn + q] == j);
      for (int q = 0; q < r; ++q) clash |= (rn_idx[p * rn + q] == js);
      pick = js;
      if (!clash) break;
    }
    rn_idx[p * rn + r] = pick;
    if (cnt) {
      const int32_t before = atomicAdd(&cnt[pick], 1);
      if (rank) rank[p * rn + r] = before;
    }
  }
}

// connected components of the undirected nn graph: parent pointers that only
// decrease, hooked across every edge and shortened by pointer jumping; at the
// fixed point every vertex points at the smallest id of its component
__global__ void cc_init_kernel(int32_t *parent, int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) parent[i] = (int32_t)i;
}

__global__ void cc_hook_kernel(const int32_t *__restrict__ nn_idx, int64_t M, int nn, int32_t *parent,
                               int32_t *changed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * nn) return;
  const int32_t j = nn_idx[e];
  if (j < 0) return;
  const int32_t pi = parent[e / nn], pj = parent[j];
  if (pi == pj) return;
  const int32_t lo = pi < pj ? pi : pj, hi = pi < pj ? pj : pi;
  atomicMin(&parent[hi], lo);
  *changed = 1;
}

__global__ void cc_shortcut_kernel(int32_t *parent, int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int32_t p = parent[i];
  int32_t gp = parent[p];
  while (p != gp) {
    p = gp;
    gp = parent[p];
  }
  parent[i] = p;
}

__global__ void inverse_perm_kernel(const int32_t *__restrict__ perm, int64_t M, int32_t *__restrict__ inv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < M) inv[perm[p]] = (int32_t)p;
}

// out[p][q] = inv[idx[perm[p]][q]] (absent slots stay -1)
__global__ void map_lists_kernel(const int32_t *__restrict__ idx, int64_t M, int k, const int32_t *__restrict__ perm,
                                 const int32_t *__restrict__ inv, int32_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  const int64_t p = e / k;
  const int q = (int)(e % k);
  const int32_t j = idx[(int64_t)perm[p] * k + q];
  out[e] = j < 0 ? -1 : inv[j];
}

// out[i][q] = perm[lists[inv[i]][q]] (back to the caller's ids and order)
__global__ void unmap_lists_kernel(const int32_t *__restrict__ lists, int64_t M, int k,
                                   const int32_t *__restrict__ perm, const int32_t *__restrict__ inv,
                                   int32_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  const int64_t i = e / k;
  const int q = (int)(e % k);
  const int32_t v = lists[(int64_t)inv[i] * k + q];
  out[e] = v < 0 ? -1 : perm[v];
}

// dst[p] = src[idx[p]] for float2 rows
__global__ void gather_f2_kernel(const float2 *__restrict__ src, const int32_t *__restrict__ idx, int64_t M,
                                 float2 *__restrict__ dst) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < M) dst[p] = src[idx ? (int64_t)idx[p] : p];
}

// flags[FLAG_BAD_INDEX] = 1 if an entry is outside [0, hi)
__global__ void range_check_kernel(const int32_t *__restrict__ idx, int64_t n, int32_t hi, int32_t *flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t j = idx[e];
  if (j < 0 || j >= hi) flags[FLAG_BAD_INDEX] = 1;
}

// reverse-neighbour mask: nn edge i -> j kept when i is among the kh helper
// neighbours of j, else -1 (absent slots stay absent)
__global__ void rnn_mask_kernel(const int32_t *nn_idx, int64_t M, int nn, const int32_t *__restrict__ helper,
                                int kh, int32_t *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * nn) return;
  const int32_t i = (int32_t)(e / nn);
  const int32_t j = nn_idx[e];
  bool keep = false;
  if (j >= 0)
    for (int r = 0; r < kh; ++r) keep |= helper[(int64_t)j * kh + r] == i;
  out[e] = keep ? j : -1;
}

__global__ void count_kernel(const int32_t *__restrict__ idx, int64_t M, int k, int32_t *cnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  int32_t j = idx[e];
  if (j >= 0) atomicAdd(&cnt[j], 1);
}

// exclusive scan of one value per thread over the block; returns the prefix
// and the block total.  256 threads = 4 waves of 64.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t val, int32_t *lds, int32_t &total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  int32_t x = val;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int32_t before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    int32_t t = lds[w];
    if (w < wid) before += t;
    total += t;
  }
  __syncthreads();
  return before + x - val;
}

__global__ void __launch_bounds__(kBlock) scan_partials_kernel(const int32_t *__restrict__ cnt,
                                                               int64_t n, int32_t *part) {
  __shared__ int32_t lds[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t idx = base + r * kBlock + threadIdx.x;
    if (idx < n) s += cnt[idx];
  }
  int32_t total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one block: exclusive scan of the nb partials in place; part[nb] = total
__global__ void __launch_bounds__(kBlock) scan_top_kernel(int32_t *part, int64_t nb) {
  __shared__ int32_t lds[kBlock / 64];
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kBlock) {
    int64_t idx = base + threadIdx.x;
    int32_t v = idx < nb ? part[idx] : 0;
    int32_t total;
    int32_t ex = block_exclusive_scan(v, lds, total);
    if (idx < nb) part[idx] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

__global__ void __launch_bounds__(kBlock) scan_final_kernel(int32_t *cnt, int64_t n,
                                                            const int32_t *__restrict__ part,
                                                            int64_t nb, int32_t *ptr) {
  __shared__ int32_t lds[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t carry = part[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t idx = base + r * kBlock + threadIdx.x;
    int32_t v = idx < n ? cnt[idx] : 0;
    int32_t total;
    int32_t ex = block_exclusive_scan(v, lds, total);
    if (idx < n) {
      ptr[idx] = carry + ex;
      cnt[idx] = carry + ex;   // cursor for the scatter
    }
    carry += total;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ptr[n] = part[nb];
}

__global__ void scatter_kernel(const int32_t *__restrict__ idx, int64_t M, int k,
                               int32_t *cursor, int32_t *__restrict__ tmp) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  int32_t j = idx[e];
  if (j < 0) return;
  int32_t slot = atomicAdd(&cursor[j], 1);
  tmp[slot] = (int32_t)(e / k);
}

// tmp[ptr[j] + rank[e]] = e / k for every edge e -> j (slots distinct by
// construction of the ranks)
__global__ void place_kernel(const int32_t *__restrict__ idx, int64_t M, int k, const int32_t *__restrict__ ptr,
                             const int32_t *__restrict__ rank, int32_t *__restrict__ tmp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  const int32_t j = idx[e];
  if (j < 0) return;
  tmp[ptr[j] + rank[e]] = (int32_t)(e / k);
}

__global__ void sort_small_kernel(const int32_t *__restrict__ ptr, const int32_t *__restrict__ tmp,
                                  int64_t M, int32_t *__restrict__ big, int32_t *flags,
                                  int32_t *__restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int32_t s = ptr[j], e = ptr[j + 1];
  const int32_t d = e - s;
  if (d > kSmallSegment) {
    int32_t pos = atomicAdd(&flags[FLAG_BIG_COUNT], 1);
    big[pos] = (int32_t)j;
    return;
  }
  // insertion sort of the segment, read from tmp, built in out
  for (int32_t p = 0; p < d; ++p) {
    int32_t x = tmp[s + p];
    int32_t q = p;
    while (q > 0) {
      int32_t w = out[s + q - 1];
      if (w <= x) break;
      out[s + q] = w;
      --q;
    }
    out[s + q] = x;
  }
}

__global__ void __launch_bounds__(kBlock) sort_big_kernel(const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ tmp,
                                                          const int32_t *__restrict__ big,
                                                          const int32_t *__restrict__ flags,
                                                          int32_t *out) {
  const int32_t nbig = flags[FLAG_BIG_COUNT];
  for (int32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int32_t j = big[b];
    const int32_t s = ptr[j];
    const int32_t d = ptr[j + 1] - s;
    int32_t *a = out + s;
    for (int32_t p = threadIdx.x; p < d; p += blockDim.x) a[p] = tmp[s + p];
    __syncthreads();
    int32_t P = 1;
    while (P < d) P <<= 1;
    for (int32_t k = 2; k <= P; k <<= 1) {
      for (int32_t jj = k >> 1; jj > 0; jj >>= 1) {
        for (int32_t i = threadIdx.x; i < P; i += blockDim.x) {
          int32_t l = (jj == (k >> 1)) ? (i ^ (k - 1)) : (i ^ jj);
          if (l > i && l < d) {
            int32_t x = a[i], y = a[l];
            if (y < x) { a[i] = y; a[l] = x; }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_validate_idx(const int32_t *idx, int64_t M, int k, int32_t lo, int32_t *flags,
                              hipStream_t s) {
  if (k == 0) return hipSuccess;
  validate_idx_kernel<<<grid_for(M * k), kBlock, 0, s>>>(idx, M, k, lo, flags);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s) {
  fill_i32_kernel<<<grid_for(n), kBlock, 0, s>>>(p, n, value);
  return hipGetLastError();
}

hipError_t launch_epoch_begin(int64_t *epoch, int32_t *cnt, int64_t M, int32_t *flags, hipStream_t s) {
  epoch_begin_kernel<<<cnt ? grid_for(M + 1) : 1, kBlock, 0, s>>>(epoch, cnt, M, flags);
  return hipGetLastError();
}

hipError_t launch_rn_sample(const int32_t *nn_idx, int64_t M, int nn, int rn, uint64_t seed,
                            const int64_t *epoch, const int32_t *perm, const int32_t *inv, int32_t *rn_idx,
                            int32_t *cnt, int32_t *rank, hipStream_t s) {
  if (rn == 0) return hipSuccess;
  rn_sample_kernel<<<grid_for(M), kBlock, 0, s>>>(nn_idx, M, nn, rn, seed, epoch, perm, inv, rn_idx, cnt, rank);
  return hipGetLastError();
}

hipError_t launch_cc_init(int32_t *parent, int64_t M, hipStream_t s) {
  cc_init_kernel<<<grid_for(M), kBlock, 0, s>>>(parent, M);
  return hipGetLastError();
}

hipError_t launch_cc_round(const int32_t *nn_idx, int64_t M, int nn, int32_t *parent, int32_t *changed,
                           hipStream_t s) {
  cc_hook_kernel<<<grid_for(M * nn), kBlock, 0, s>>>(nn_idx, M, nn, parent, changed);
  cc_shortcut_kernel<<<grid_for(M), kBlock, 0, s>>>(parent, M);
  return hipGetLastError();
}

hipError_t launch_inverse_perm(const int32_t *perm, int64_t M, int32_t *inv, hipStream_t s) {
  inverse_perm_kernel<<<grid_for(M), kBlock, 0, s>>>(perm, M, inv);
  return hipGetLastError();
}

hipError_t launch_map_lists(const int32_t *idx, int64_t M, int k, const int32_t *perm, const int32_t *inv,
                            int32_t *out, hipStream_t s) {
  if (k == 0) return hipSuccess;
  map_lists_kernel<<<grid_for(M * k), kBlock, 0, s>>>(idx, M, k, perm, inv, out);
  return hipGetLastError();
}

hipError_t launch_unmap_lists(const int32_t *lists, int64_t M, int k, const int32_t *perm, const int32_t *inv,
                              int32_t *out, hipStream_t s) {
  if (k == 0) return hipSuccess;
  unmap_lists_kernel<<<grid_for(M * k), kBlock, 0, s>>>(lists, M, k, perm, inv, out);
  return hipGetLastError();
}

__global__ void probe_atomic_kernel(uint64_t *acc, const int32_t *__restrict__ idx, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) atomicAdd((unsigned long long *)(acc + idx[t]), (1ull << 32) | 1ull);
}

hipError_t launch_probe_atomic(uint64_t *acc, const int32_t *idx, int64_t n, hipStream_t s) {
  probe_atomic_kernel<<<grid_for(n), kBlock, 0, s>>>(acc, idx, n);
  return hipGetLastError();
}

hipError_t launch_gather_f2(const float2 *src, const int32_t *idx, int64_t M, float2 *dst, hipStream_t s) {
  gather_f2_kernel<<<grid_for(M), kBlock, 0, s>>>(src, idx, M, dst);
  return hipGetLastError();
}

hipError_t launch_rnn_mask(const int32_t *nn_idx, int64_t M, int nn, const int32_t *helper, int kh, int32_t *out,
                           hipStream_t s) {
  rnn_mask_kernel<<<grid_for(M * nn), kBlock, 0, s>>>(nn_idx, M, nn, helper, kh, out);
  return hipGetLastError();
}

hipError_t launch_count(const int32_t *idx, int64_t M, int k, int32_t *cnt, hipStream_t s) {
  if (k == 0) return hipSuccess;
  count_kernel<<<grid_for(M * k), kBlock, 0, s>>>(idx, M, k, cnt);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t *cnt, int64_t M, int32_t *part, int32_t *ptr, hipStream_t s) {
  const int64_t nb = (M + kScanChunk - 1) / kScanChunk;
  scan_partials_kernel<<<(unsigned)nb, kBlock, 0, s>>>(cnt, M, part);
  scan_top_kernel<<<1, kBlock, 0, s>>>(part, nb);
  scan_final_kernel<<<(unsigned)nb, kBlock, 0, s>>>(cnt, M, part, nb, ptr);
  return hipGetLastError();
}

hipError_t launch_range_check(const int32_t *idx, int64_t n, int32_t hi, int32_t *flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  range_check_kernel<<<grid_for(n), kBlock, 0, s>>>(idx, n, hi, flags);
  return hipGetLastError();
}

hipError_t launch_transpose(const int32_t *idx, int64_t rows, int k, int64_t ntargets, int32_t *ptr, int32_t *cnt,
                            int32_t *part, int32_t *tmp, int32_t *big, int32_t *flags, int32_t *src_out,
                            hipStream_t s) {
  fill_i32_kernel<<<grid_for(ntargets + 1), kBlock, 0, s>>>(cnt, ntargets + 1, 0);
  fill_i32_kernel<<<1, kBlock, 0, s>>>(flags + FLAG_BIG_COUNT, 1, 0);
  count_kernel<<<grid_for(rows * k), kBlock, 0, s>>>(idx, rows, k, cnt);
  hipError_t e = launch_scan(cnt, ntargets, part, ptr, s);
  if (e != hipSuccess) return e;
  scatter_kernel<<<grid_for(rows * k), kBlock, 0, s>>>(idx, rows, k, cnt, tmp);
  sort_small_kernel<<<grid_for(ntargets), kBlock, 0, s>>>(ptr, tmp, ntargets, big, flags, src_out);
  sort_big_kernel<<<kBigSortBlocks, kBlock, 0, s>>>(ptr, tmp, big, flags, src_out);
  return hipGetLastError();
}

hipError_t launch_place_sort(const int32_t *idx, int64_t M, int k, const int32_t *ptr, const int32_t *rank,
                             int32_t *tmp, int32_t *big, int32_t *flags, int32_t *src_out, hipStream_t s) {
  if (k == 0) return hipSuccess;
  place_kernel<<<grid_for(M * k), kBlock, 0, s>>>(idx, M, k, ptr, rank, tmp);
  sort_small_kernel<<<grid_for(M), kBlock, 0, s>>>(ptr, tmp, M, big, flags, src_out);
  sort_big_kernel<<<kBigSortBlocks, kBlock, 0, s>>>(ptr, tmp, big, flags, src_out);
  return hipGetLastError();
}

hipError_t launch_scatter_sort(const int32_t *idx, int64_t M, int k, const int32_t *ptr,
                               int32_t *cursor, int32_t *tmp, int32_t *big, int32_t *flags,
                               int32_t *src_out, hipStream_t s) {
  if (k == 0) return hipSuccess;
  scatter_kernel<<<grid_for(M * k), kBlock, 0, s>>>(idx, M, k, cursor, tmp);
  sort_small_kernel<<<grid_for(M), kBlock, 0, s>>>(ptr, tmp, M, big, flags, src_out);
  sort_big_kernel<<<kBigSortBlocks, kBlock, 0, s>>>(ptr, tmp, big, flags, src_out);
  return hipGetLastError();
}

}  // namespace ivhd
