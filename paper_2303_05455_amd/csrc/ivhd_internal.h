// Internal declarations shared by the HIP translation units of libivhd.
// Not part of the public ABI (that is include/ivhd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ivhd.h"

namespace ivhd {

constexpr int kBlock = 256;          // threads per block of the per-vertex kernels
constexpr int kScanItems = 8;        // items per thread in the block scan
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kSmallSegment = 32;    // in-edge segments up to this size are sorted per thread
constexpr int kBigSortBlocks = 256;  // blocks that share the list of large segments
constexpr int kHeavyDegree = 80;     // nn in-degree above which a vertex gets a whole wavefront (large graphs)
constexpr int kSmallGraphHeavyDegree = 16;   // the same below kSmallGraphVertices
constexpr int64_t kSmallGraphVertices = 500000;
constexpr int kSmallGraphLanes = 4;  // lanes per light vertex of the deterministic step below that size
constexpr int kDetBlock = 64;        // threads per block of the deterministic step kernel (one wavefront)
constexpr int kHeavyPerBlock = kDetBlock / 64;
constexpr int kXcds = 8;             // MI355X: 8 XCDs, workgroups dealt round-robin

// device flag slots
enum { FLAG_BAD_INDEX = 0, FLAG_NONFINITE = 1, FLAG_BIG_COUNT = 2, FLAG_SLOTS = 4 };

// error reporting shared by the host translation units (message is thread-local)
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return ::ivhd::hip_fail(_e, #expr); \
  } while (0)

template <typename T>
int dev_alloc(T **p, size_t count, const char *what) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? IVHD_ENOMEM : IVHD_EDEVICE, "allocating %s (%zu bytes): %s", what,
                count * sizeof(T), hipGetErrorString(e));
  }
  return IVHD_OK;
}

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// Transposed (CSC) edge lists: for every target j, the sources s of the
// edges s -> j, sorted ascending (multiplicity kept).
struct Csc {
  int32_t *ptr = nullptr;   // [M+1]
  int32_t *src = nullptr;   // [capacity]
};

// Scratch shared by CSC builds.
struct CscScratch {
  int32_t *cnt = nullptr;        // [M+1]: counts, then the scatter cursor
  int32_t *tmp = nullptr;        // [capacity]: unsorted sources
  int32_t *part = nullptr;       // [ceil((M+1)/kScanChunk)] block partial sums
  int32_t *big = nullptr;        // [M]: targets with a segment above kSmallSegment
  int32_t *rank = nullptr;       // [M*rn]: each rn draw's arrival rank among its target's in-edges
};

// ---- graph.hip ----
// flags[FLAG_BAD_INDEX] = 1 if an entry is outside [lo, M) or equals its row (lo = -1 allows absent slots)
hipError_t launch_validate_idx(const int32_t *idx, int64_t M, int k, int32_t lo, int32_t *flags, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s);
// Begins a random-neighbour epoch: epoch += 1; when cnt != NULL zeroes cnt[0..M] and flags[FLAG_BIG_COUNT].
hipError_t launch_epoch_begin(int64_t *epoch, int32_t *cnt, int64_t M, int32_t *flags, hipStream_t s);
// rn draw for epoch *epoch (caller ids; with perm/inv stored as internal ids in
// internal row order); when cnt != NULL also counts in-degrees into cnt and,
// when rank != NULL, stores each draw's arrival rank at its target (the
// count before it).
hipError_t launch_rn_sample(const int32_t *nn_idx, int64_t M, int nn, int rn, uint64_t seed,
                            const int64_t *epoch, const int32_t *perm, const int32_t *inv, int32_t *rn_idx,
                            int32_t *cnt, int32_t *rank, hipStream_t s);
// connected components (parent -> smallest id of the component)
hipError_t launch_cc_init(int32_t *parent, int64_t M, hipStream_t s);
hipError_t launch_cc_round(const int32_t *nn_idx, int64_t M, int nn, int32_t *parent, int32_t *changed,
                           hipStream_t s);
hipError_t launch_inverse_perm(const int32_t *perm, int64_t M, int32_t *inv, hipStream_t s);
hipError_t launch_map_lists(const int32_t *idx, int64_t M, int k, const int32_t *perm, const int32_t *inv,
                            int32_t *out, hipStream_t s);
hipError_t launch_unmap_lists(const int32_t *lists, int64_t M, int k, const int32_t *perm, const int32_t *inv,
                              int32_t *out, hipStream_t s);
hipError_t launch_gather_f2(const float2 *src, const int32_t *idx, int64_t M, float2 *dst, hipStream_t s);
// acc[idx[t]] += 2^32 + 1 for t < n, one 64-bit integer atomic each (a rate probe)
hipError_t launch_probe_atomic(uint64_t *acc, const int32_t *idx, int64_t n, hipStream_t s);
// out[i][q] = nn_idx[i][q] when i is among helper[j][0..kh) for j = nn_idx[i][q] >= 0, else -1
hipError_t launch_rnn_mask(const int32_t *nn_idx, int64_t M, int nn, const int32_t *helper, int kh, int32_t *out,
                           hipStream_t s);
// in-degree count of an [M][k] index list (entries < 0 skipped); cnt must be zero.
hipError_t launch_count(const int32_t *idx, int64_t M, int k, int32_t *cnt, hipStream_t s);
// From counts cnt[0..M-1]: ptr = exclusive scan (ptr[M] = total), cnt = cursor copy.
hipError_t launch_scan(int32_t *cnt, int64_t M, int32_t *part, int32_t *ptr, hipStream_t s);
// flags[FLAG_BAD_INDEX] = 1 if an entry of idx[0..n) is outside [0, hi)
hipError_t launch_range_check(const int32_t *idx, int64_t n, int32_t hi, int32_t *flags, hipStream_t s);
// Transpose of rows x k lists with targets in [0, ntargets) (entries < 0 skipped): ptr [ntargets+1],
// src_out [rows*k] (per target the source rows ascending).  Scratch: cnt [ntargets+1], part
// [ntargets / kScanChunk + 2], tmp [rows*k], big [ntargets].
hipError_t launch_transpose(const int32_t *idx, int64_t rows, int k, int64_t ntargets, int32_t *ptr, int32_t *cnt,
                            int32_t *part, int32_t *tmp, int32_t *big, int32_t *flags, int32_t *src_out,
                            hipStream_t s);
// Placement by arrival rank (tmp[ptr[j] + rank[e]] = source of edge e, no
// atomics) + canonical sort: src_out segments end sorted ascending.
hipError_t launch_place_sort(const int32_t *idx, int64_t M, int k, const int32_t *ptr, const int32_t *rank,
                             int32_t *tmp, int32_t *big, int32_t *flags, int32_t *src_out, hipStream_t s);
// Scatter + canonical sort: csc.src segments end sorted ascending.
hipError_t launch_scatter_sort(const int32_t *idx, int64_t M, int k, const int32_t *ptr,
                               int32_t *cursor, int32_t *tmp, int32_t *big, int32_t *flags,
                               int32_t *src_out, hipStream_t s);

// ---- order.hip ----
// perm = the ids 0..M-1 sorted by (root[i], min(indeg[i], heavy_deg + 1),
// first nn neighbour of i (absent last), i); nn_idx is [M, nn] with nn >= 1;
// synchronises s
int sort_vertex_order(const int32_t *root, const int32_t *indeg, const int32_t *nn_idx, int nn, int64_t M,
                      int heavy_deg, int32_t *perm, hipStream_t s);
// the whole order: components of the undirected nn graph (at most
// kCcMaxRounds rounds), in-degrees, the sort above, and inv = perm^-1.
// parent [M] and indeg [M+1] are scratch, changed one device int;
// synchronises s
constexpr int kCcMaxRounds = 64;   // pointer jumping converges long before
int build_vertex_order(const int32_t *nn_idx, int64_t M, int nn, int heavy_deg, int32_t *parent, int32_t *indeg,
                       int32_t *changed, int32_t *perm, int32_t *inv, hipStream_t s);

// ---- step.hip ----
// device state of the self-adaptive b
struct AdaptState {
  float b;            // current step factor
  int32_t reject;     // 1: the last tentative step was rejected
  int64_t kept, rejected;
  double dT;          // kinetic energy change of the last tentative step
};

// state of Adam on the loop: step count and bias corrections of this step
struct AdamState {
  int64_t t;
  float c1, c2;       // 1 - beta1^t, 1 - beta2^t
};

// update rule of the deterministic step (template argument of its kernel)
enum { OPT_PLAIN = 0, OPT_NEST = 1, OPT_ADAPT = 2, OPT_ADAM = 3 };

// Atomic mode: the rn reactions a vertex receives are summed in fixed point,
// x and y as two signed 32-bit fields of one 64-bit integer, so that one
// integer atomic carries both coordinates and the sum does not depend on the
// order of arrival.  The unit is c 2^-kReactionFracBits; after each draw the
// range of one reaction is set to 2^e units with e = 30 - ceil(log2 K), K the
// largest rn in-degree of the draw, so no field's sum can leave
// [-2^30, 2^30].  Reactions outside the range go to a float accumulator.
constexpr int kReactionFracBits = 22;
constexpr int kRangeParts = 256;   // blocks of the in-degree maximum
struct ReactionRange {
  int32_t part[kRangeParts];   // per-block maxima of the in-degree
  float cap;                   // largest |reaction| / unit held in fixed point (a power of two)
};
// rr->cap from the rn in-degree counts cnt[0..M) of a draw (two kernels)
hipError_t launch_reaction_range(const int32_t *cnt, int64_t M, ReactionRange *rr, hipStream_t s);

struct StepArgs {
  const float2 *y;        // positions read (Y_n)
  const float2 *h;        // positions the forces are taken at: y, or H = Y + a V (nesterov)
  float2 *y_out;          // positions written (Y_{n+1}); det mode: != y
  float2 *h_out;          // nesterov: H_{n+1} written here
  float2 *v;              // velocities, in place (read only with adapt)
  float2 *v_out;          // adapt: tentative velocities
  const float *b_dev;     // adapt: b read from device memory
  double *ke_part;        // adapt: per-block sums of |v'|^2 - |v|^2 [det_grid]
  float2 *s2;             // adam: second moments (v holds the first moments)
  const AdamState *adam;  // adam: bias corrections of this step
  float lr, beta1, beta2, eps_adam;
  int32_t l1, opt;        // opt: OPT_* (atomic mode: OPT_PLAIN or OPT_NEST)
  const int32_t *nn_idx;  // [M][nn]
  const int32_t *rn_idx;  // [M][rn]
  const int32_t *nn_ptr, *nn_src;   // CSC of nn edges
  const int32_t *rn_ptr, *rn_src;   // CSC of rn edges
  float2 *fbuf;           // atomic mode: float accumulator of the rn reactions outside the fixed range [M]
  float2 *fown;           // atomic mode: each vertex's own share of its force [M]
  uint64_t *facc;         // atomic mode: packed fixed-point accumulator of the rn reactions [M]
  const ReactionRange *rx;   // atomic mode: the fixed-point range of the current draw
  float rx_unit, rx_inv_unit;   // atomic mode: the fixed-point unit c 2^-kReactionFracBits and its inverse
  int32_t *fflag;         // atomic mode: [2] set when a pass 1 used fbuf (slot fpar); see gather_reactions
  int32_t fpar;           // atomic mode: the slot of this iteration (alternates from one to the next)
  int32_t *flags;
  const float *gscale;    // gradient kernels: output scaled by *gscale (NULL = 1)
  const int32_t *out_perm;   // gradient kernels: vertex i's output goes to out[out_perm[i]] (NULL: out[i])
  double *e_part;         // gradient kernels: FP64 stress of each block's out-edges [det_grid] (NULL: none)
  const int32_t *heavy;   // vertices whose nn in-degree exceeds heavy_deg
  int32_t n_heavy;
  int32_t heavy_deg;      // nn in-degree above which a vertex gets a whole wavefront
  int32_t heavy_blocks;   // leading blocks of a launch that serve the heavy vertices (multiple of kXcds)
  int32_t lanes;          // lanes per light vertex: 1, or kSmallGraphLanes below kSmallGraphVertices
  int32_t light_tiles;    // tiles of kDetBlock / lanes consecutive vertices
  int32_t tiles_per_xcd;  // consecutive tiles given to each XCD
  int64_t M;
  int nn, rn;
  float a, b, c, eps;
};
// launch shape of the deterministic kernel: heavy blocks first (rounded to a
// multiple of kXcds so the round-robin phase is kept), then the light tiles,
// XCD x taking tiles [x * tiles_per_xcd, (x + 1) * tiles_per_xcd)
inline void set_launch_shape(StepArgs &a) {
  const int32_t hb = (a.n_heavy + kHeavyPerBlock - 1) / kHeavyPerBlock;
  a.heavy_blocks = (hb + kXcds - 1) / kXcds * kXcds;
  a.lanes = a.M < kSmallGraphVertices ? kSmallGraphLanes : 1;
  const int32_t per_tile = kDetBlock / a.lanes;
  a.light_tiles = (int32_t)((a.M + per_tile - 1) / per_tile);
  a.tiles_per_xcd = (a.light_tiles + kXcds - 1) / kXcds;
}
unsigned det_grid(const StepArgs &a);   // blocks of one deterministic launch
hipError_t launch_step_det(const StepArgs &a, hipStream_t s);
hipError_t launch_lookahead(const float2 *y, const float2 *v, float a, int64_t M, float2 *h, hipStream_t s);
// t += 1 and the bias corrections of step t
hipError_t launch_adam_prep(AdamState *st, float beta1, float beta2, hipStream_t s);
hipError_t launch_adapt_decide(const double *part, int nparts, double tau, float g1, float g2, AdaptState *st,
                               hipStream_t s);
// when st->reject: y_next = y, v_next = v
hipError_t launch_adapt_commit(const AdaptState *st, const float2 *y, const float2 *v, int64_t M, float2 *y_next,
                               float2 *v_next, hipStream_t s);
hipError_t launch_step_atomic(const StepArgs &a, hipStream_t s);   // two kernels
// grad E = -2 f at positions a.y into out (det gather; or the atomic mode's two passes)
hipError_t launch_grad_det(const StepArgs &a, float2 *out, hipStream_t s);
hipError_t launch_grad_atomic(const StepArgs &a, float2 *out, hipStream_t s);

// transposed lists of an [M][k] index list into g; the heavy list (synchronises s)
int build_csc(const int32_t *idx, int64_t M, int k, Csc &g, CscScratch &sc, int32_t *flags, hipStream_t s);
int build_heavy(const Csc &nn_csc, int64_t M, int heavy_deg, int32_t *heavy, int32_t *flags, int32_t *n_heavy,
                hipStream_t s);
// the hub threshold of a graph of M vertices: kHeavyDegree for large graphs;
// small graphs have too few wavefronts to hide a thread's long in-edge chain,
// so more of their vertices get a wavefront
int heavy_degree(int64_t M);
// list the vertices with nn in-degree > heavy_deg (order arbitrary); *count must be zero
hipError_t launch_heavy_list(const int32_t *nn_ptr, int64_t M, int heavy_deg, int32_t *list, int32_t *count,
                             hipStream_t s);

// ---- reduce.hip ----
// FP64 stress: per-block partial sums (fixed tree), then one block in fixed order.
// metric: 0 Euclidean, 1 l1
hipError_t launch_stress(const float2 *y, int64_t M, const int32_t *nn_idx, int nn,
                         const int32_t *rn_idx, int rn, double c, int metric, double *partials,
                         int nparts, double *out, hipStream_t s);
int stress_partials(int64_t M);
// *out = the fixed-order sum of partials[0..nparts) (one block)
hipError_t launch_stress_final(const double *partials, int nparts, double *out, hipStream_t s);
// out[k] = *scale * x[k], k < n
hipError_t launch_scale_f32(const float *x, int64_t n, const float *scale, float *out, hipStream_t s);

// ---- knn.hip ----
int knn_max_k();
hipError_t launch_row_norms(const float *X, int64_t M, int N, float *out, hipStream_t s);
// largest |X[e]| over n values as float bits, max-combined into *out (zero it first)
hipError_t launch_absmax(const float *X, int64_t n, uint32_t *out, hipStream_t s);
int knn_padded_width(int N);            // N rounded up to the staged K step
float knn_split_scale(float absmax);    // power of two keeping scaled values below 2^14
// hi / lo FP16 rows of scale * X, [M][Np], zero padded
hipError_t launch_split(const float *X, int64_t M, int N, int Np, float scale, _Float16 *hi, _Float16 *lo,
                        hipStream_t s);
// self_mode: 0 = none, 1 = query q excludes candidate q, 2 = query q excludes self[q].
// Xh/Xl, Qh/Ql: the split rows of X and Q at the same scale (Qh == Xh when Q == X).
hipError_t launch_knn(const float *X, int64_t M, int N, const float *Q, int64_t nq, const _Float16 *Xh,
                      const _Float16 *Xl, const _Float16 *Qh, const _Float16 *Ql, int Np, float scale,
                      int self_mode, const int32_t *self, const float *cnorm, int k, int32_t *idx, float *dist,
                      hipStream_t s);

// inverted-file search (knn.hip): split rows gathered in list order
hipError_t launch_gather_f32(const float *src, const int32_t *idx, int64_t n, float *dst, hipStream_t s);
hipError_t launch_split_gather(const float *X, int64_t M, int N, int Np, float scale, const int32_t *pos_id,
                               _Float16 *hi, _Float16 *lo, hipStream_t s);
// one block per work item (list work_list[b], chunk work_chunk[b] of its probing queries); each
// query's top k of the list goes to part_[idx|dist][(q * nprobe + slot) * k]
hipError_t launch_ivf_lists(const float *X, int N, const float *Q, const _Float16 *Xh, const _Float16 *Xl,
                            const _Float16 *Qh, const _Float16 *Ql, int Np, float scale, const float *pnorm,
                            const int32_t *pos_id, const int32_t *lptr, const int32_t *pptr, const int32_t *pq,
                            const int32_t *work_list, const int32_t *work_chunk, int64_t n_work,
                            const int32_t *probes, int nprobe, const int32_t *self, int k, int32_t *part_idx,
                            float *part_dist, hipStream_t s);
hipError_t launch_ivf_merge(const int32_t *part_idx, const float *part_dist, int64_t nq, int nprobe, int k,
                            int32_t *idx, float *dist, hipStream_t s);
hipError_t launch_init_centroids(const float *X, int64_t M, int N, int nlist, float *C, hipStream_t s);
hipError_t launch_centroid_mean(const float *X, int N, const int32_t *lptr, const int32_t *pos_id, int nlist,
                                float *C, hipStream_t s);

}  // namespace ivhd
