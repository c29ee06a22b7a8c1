/*
 * ivhd.h -- C ABI of the MI355X (gfx950) IVHD embedding library.
 *
 * IVHD embeds a kNN graph in 2-D.  Every vertex i has up to nn
 * nearest-neighbour out-edges O_nn(i) (target distance 0) and rn random
 * out-edges O_rn(i) (target distance 1) drawn by the library.  The layout Y
 * minimises the binary-distance stress
 *
 *     E(Y) = sum_i [ sum_{j in O_nn(i)} |y_i - y_j|^2
 *                    + c * sum_{k in O_rn(i)} (1 - |y_i - y_k|)^2 ]
 *
 * (thesis: Sec. "Improving classical MDS", Eq. ivhd_cost_function with the
 * binary dissimilarities of Eq. ivhd_binary_distances) by the damped
 * particle method of Sec. "Force directed", Eq. force_directed_update:
 *
 *     f  = -1/2 grad E        (every edge acts on both of its ends)
 *     V <- a V + b f ;  Y <- Y + V      (all vertices from the same Y)
 *
 * Conventions shared by every entry point
 *  - All pointers named d_* are HIP device pointers on the current device,
 *    owned by the CALLER, contiguous, row-major.  h_* are host pointers.
 *  - Positions and velocities are float32 [M][2] (x, y interleaved).
 *  - Vertex ids are int32; a neighbour slot holding -1 is absent (a vertex
 *    with fewer than nn neighbours keeps all it has, Sec. "Force directed").
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls return before the GPU finishes unless the
 *    entry point says it synchronises.
 *  - Every call returns an ivhd_status.  Nothing is thrown or aborted across
 *    the ABI.  On failure ivhd_last_error() holds a message (thread-local,
 *    valid until the next call on that thread).  Arguments are validated on
 *    the host before any device work, so an IVHD_EINVAL from validation
 *    leaves device memory untouched.
 */
#ifndef IVHD_H
#define IVHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ivhd_status {
    IVHD_OK = 0,
    IVHD_EINVAL = -1,    /* bad argument, or (at init) a bad neighbour index */
    IVHD_ENOMEM = -2,    /* device allocation failed */
    IVHD_EDEVICE = -3,   /* a HIP call failed */
    IVHD_ESTATE = -4,    /* NULL or destroyed context */
    IVHD_ENUMERIC = -5   /* a non-finite position or force was produced */
} ivhd_status;

typedef enum ivhd_mode {
    IVHD_MODE_DET = 0,     /* per-vertex gather over out-edges and transposed
                              in-edges, fixed order, no atomics: bitwise
                              reproducible run to run                        */
    IVHD_MODE_ATOMIC = 1   /* a pass that gathers each vertex's nn edges (both
                              ways) and rn out-edges, adding each rn edge's
                              reaction to the other end with one 64-bit
                              integer atomic (x and y in fixed point, unit
                              c 2^-22, range set after each draw from the
                              largest rn in-degree), then an update pass.
                              Integer sums do not depend on the order of
                              arrival: bitwise reproducible run to run, unless
                              a reaction exceeds the fixed-point range (then
                              it goes through float atomics, whose order of
                              summation varies)                             */
} ivhd_mode;

/* ivhd_params.flags */
#define IVHD_FLAG_REORDER 1   /* keep the vertices internally grouped by connected
                                 component of the nn graph (smallest id first), and
                                 inside a component by nn in-degree capped at 81
                                 (17 below 500,000 vertices), then by first nn
                                 neighbour (absent last), then by id (a
                                 locality and load-balance order; the
                                 results are the same up to floating-point summation
                                 order, and the caller always sees its own order)  */
#define IVHD_FLAG_NESTEROV 2  /* Nesterov momentum (Sec. "Optimization methods"): the
                                 force of each step is taken at the look-ahead layout
                                 H = Y + a V,  V <- a V + b f(H),  Y <- Y + V.  One
                                 more (det: two more) [M][2] float buffers.        */
#define IVHD_FLAG_L1 4        /* the l1 distance d = |dx| + |dy| in the stress and
                                 its force (Sec. "L1 norm in late stages of
                                 embedding"); the force is -1/2 grad E with
                                 sign(0) = 0.  ivhd_stress / ivhd_grad of the
                                 context use the same distance.                    */

typedef struct ivhd_params {
    int64_t  M;       /* vertices; 2 <= M <= 2^31 - 2                        */
    int32_t  nn;      /* nn slots per vertex, 1..64                          */
    int32_t  rn;      /* random neighbours per vertex, 0..64; nn + rn <= M-1 */
    float    a;       /* momentum (friction) factor, 0 <= a <= 1             */
    float    b;       /* force step, b > 0                                   */
    float    c;       /* random-edge weight, 0 < c < 1                       */
    float    eps;     /* guard of the rn unit vector y_ik / max(d, eps); >= 0 */
    uint64_t seed;    /* random-neighbour generator key                       */
    int32_t  rn_resample_every; /* R: draw new random neighbours at every
                                   iteration n with n % R == 0; 0 = draw once */
    int32_t  mode;    /* ivhd_mode                                            */
    int32_t  flags;   /* IVHD_FLAG_* bits                                     */
    int32_t  reserved;/* must be 0                                            */
} ivhd_params;

typedef struct ivhd_ctx ivhd_ctx;   /* opaque */

/* Random-neighbour draw (the rule of Sec. "Improving classical MDS": rn
 * random non-neighbours per vertex, generated ad hoc; Sec. "Force directed":
 * a connected neighbour is never a random one).  For epoch e, vertex i, slot
 * r and try t = 0..255:
 *     ctr = ((e*M + i)*rn + r)*256 + t
 *     h   = splitmix64(seed ^ splitmix64(ctr))       (SplitMix64, Steele et al. 2014)
 *     j   = h mod (M-1); if (j >= i) j += 1
 * the try is rejected if j is in O_nn(i) or already drawn for i; try 255 is
 * accepted whatever it gives.  Epoch e covers iterations [e*R, (e+1)*R).   */

/* ivhd_init: create a context for one graph and one layout.
 *   d_nn_idx  int32 [M][nn], read at init and at every random-neighbour draw;
 *             must stay valid and unchanged for the context's lifetime.
 *   d_y, d_v  float32 [M][2], the initial positions and velocities (d_v is
 *             normally zeros).  The context copies them into its own buffers
 *             and writes the state back into them at the end of every
 *             ivhd_step; they must stay valid for the context's lifetime.
 *             Changes the caller makes to them are not read back (see
 *             ivhd_set_state).
 *   stream    hipStream_t all later calls enqueue on.
 * Draws the random neighbours of epoch 0, builds the internal vertex order
 * (IVHD_FLAG_REORDER) and the transposed edge lists.  Synchronises `stream`.
 * Returns IVHD_EINVAL (and no context) when an nn entry is outside [-1, M)
 * or equals its own row.                                                    */
int ivhd_init(ivhd_ctx **out, const ivhd_params *p, const int32_t *d_nn_idx,
              float *d_y, float *d_v, void *stream);

/* ivhd_step: n_iters >= 0 iterations of the loop; asynchronous.  Y and V are
 * written back to the caller's buffers (in the caller's order) at the end.
 * Iterations are replayed from captured HIP graphs when possible (one graph
 * per random-neighbour epoch).                                              */
int ivhd_step(ivhd_ctx *ctx, int64_t n_iters);

/* ivhd_set_state: load positions and velocities (float32 [M][2] each, the
 * caller's order) into the context, e.g. to resume from a checkpoint.
 * Asynchronous.                                                             */
int ivhd_set_state(ivhd_ctx *ctx, const float *d_y, const float *d_v);

/* ivhd_set_iteration: set the iteration counter to n and redraw the random
 * neighbours held before iteration n (epoch (n-1)/R, epoch 0 when n = 0 or
 * R = 0).  With ivhd_set_state this resumes a run exactly: a checkpoint is
 * (Y, V, n) and the parameters.  Synchronises the stream.                   */
int ivhd_set_iteration(ivhd_ctx *ctx, int64_t n);

/* ivhd_stress: E(Y) accumulated in FP64 from the FP32 positions, with a
 * fixed-order (deterministic) reduction.  d_y = NULL uses the context's Y;
 * otherwise float32 [M][2] evaluated with the context's current edges.
 * Synchronises the stream.  IVHD_ENUMERIC if E is not finite.             */
int ivhd_stress(ivhd_ctx *ctx, const float *d_y, double *h_E);

/* ivhd_grad: d_grad = grad E (= -2 f) in FP32, float32 [M][2]; d_y as in
 * ivhd_stress.  Asynchronous.                                               */
int ivhd_grad(ivhd_ctx *ctx, const float *d_y, float *d_grad);

/* ivhd_get_rn: copy the current epoch's random neighbours, int32 [M][rn]. */
int ivhd_get_rn(ivhd_ctx *ctx, int32_t *d_rn_out);

/* ivhd_get_in_edges: copy the transposed (in-edge) lists the deterministic
 * mode gathers over: which = 0 for the nn edges, 1 for the current epoch's
 * rn edges.  d_ptr int32 [M+1] (offsets), d_src int32 [M*nn] or [M*rn]
 * (sources of the edges into each vertex, ascending; only the first
 * d_ptr[M] entries are written).  Vertices are numbered in the internal
 * order (ivhd_get_order).  IVHD_EINVAL in atomic mode for which = 1 (that
 * mode keeps no rn in-edge lists).                                          */
int ivhd_get_in_edges(ivhd_ctx *ctx, int32_t which, int32_t *d_ptr, int32_t *d_src);

/* ivhd_get_order: d_perm int32 [M]: the caller's id of internal vertex p
 * (the identity without IVHD_FLAG_REORDER).                                 */
int ivhd_get_order(ivhd_ctx *ctx, int32_t *d_perm);

/* ivhd_get_iteration: the number of iterations done so far.                */
int ivhd_get_iteration(const ivhd_ctx *ctx, int64_t *h_n);

/* ivhd_set_graphs: 1 = replay captured HIP graphs (default), 0 = launch each
 * kernel directly.  Results are identical either way.                       */
int ivhd_set_graphs(ivhd_ctx *ctx, int32_t enable);

/* ivhd_set_adaptive: the self-adaptive b of Sec. "Force directed".  With
 * enable = 1 every iteration is tentative: V' = a V + b f, Y' = Y + V', and
 * with dT = sum_i |V'_i|^2 - |V_i|^2 (FP64 sum) the step is kept when dT is
 * finite and |dT| <= tau; otherwise Y and V stay as they were and b is
 * scaled by g1 (dT < -tau) or g2 (dT > tau or not finite).  Rejected steps
 * still count as iterations (they advance the random-neighbour schedule).
 *   b     the current b (replaces params.b), b > 0
 *   tau   threshold on |dT|, tau >= 0 (+inf: never reject)
 *   g1    > 1;  g2 in (0, 1)
 * Deterministic mode only, not with IVHD_FLAG_NESTEROV or Adam (IVHD_EINVAL).
 * Clears the kept / rejected counters.  enable = 0 returns to the fixed
 * params.b (the other arguments are ignored).  Synchronises the stream.     */
int ivhd_set_adaptive(ivhd_ctx *ctx, int32_t enable, float b, double tau, float g1, float g2);

/* ivhd_set_adam: Adam (Sec. "Optimization methods") in place of the momentum
 * update, on the gradient g = grad E per coordinate:
 *   m <- beta1 m + (1 - beta1) g,  s <- beta2 s + (1 - beta2) g^2,
 *   Y <- Y - lr (m / (1 - beta1^t)) / (eps + sqrt(s / (1 - beta2^t))),
 * t = 1, 2, ... counting Adam steps since it was enabled.  V holds (and
 * returns to the caller) the first moments m.  enable = 1 zeroes m and s
 * and restarts t; enable = 0 goes back to the momentum update with the
 * current V.  lr > 0, beta1 and beta2 in [0, 1), eps > 0.  Deterministic
 * mode only, not with IVHD_FLAG_NESTEROV or the adaptive b (IVHD_EINVAL).
 * Synchronises the stream.                                                  */
int ivhd_set_adam(ivhd_ctx *ctx, int32_t enable, float lr, float beta1, float beta2, float eps);

/* ivhd_get_adaptive: the adaptive state after the work queued so far
 * (synchronises): current b, kept and rejected step counts, and dT of the
 * last tentative step.  Any output pointer may be NULL.  IVHD_EINVAL if the
 * adaptive b was never enabled on this context.                             */
int ivhd_get_adaptive(ivhd_ctx *ctx, float *h_b, int64_t *h_kept, int64_t *h_rejected, double *h_dT);

/* ivhd_destroy: free everything the context owns (not the caller's buffers).
 * Synchronises the stream.  NULL is accepted.                               */
int ivhd_destroy(ivhd_ctx *ctx);

/* ---- the stress as a differentiable function of the layout ---------------
 * An edge plan holds the transposed lists of caller-given nn and rn edge
 * lists so that the stress E(Y) of Eq. ivhd_cost_function and its gradient
 * can be evaluated for many layouts Y (a loss for gradient-based training).
 * Without IVHD_EDGES_REORDER the plan keeps the caller's index pointers:
 * they must then stay valid and unchanged while the plan lives. */
typedef struct ivhd_edges ivhd_edges;   /* opaque */

/* ivhd_edges_create: d_nn_idx int32 [M][nn], d_rn_idx int32 [M][rn] (-1 =
 * absent slot in either), rn may be 0 (d_rn_idx ignored).
 * Entries equal to their own row are rejected (IVHD_EINVAL).  flags: 0 or
 * IVHD_EDGES_REORDER, which makes the plan keep its own copy of the lists in
 * the internal vertex order of IVHD_FLAG_REORDER; every stress and gradient
 * call then gathers Y into that order first (one extra pass over Y, paid
 * back by the locality of the edge gathers on large graphs; results equal
 * up to floating-point summation order, inputs and outputs in the caller's
 * order).  Building the order costs a few milliseconds at a million
 * vertices.  Other bits: IVHD_EINVAL.  Synchronises the stream; the plan's
 * later calls run on this stream.                                          */
#define IVHD_EDGES_REORDER 1
int ivhd_edges_create(ivhd_edges **out, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                      const int32_t *d_rn_idx, int32_t rn, int32_t flags, void *stream);

/* ivhd_edges_stress: *d_E (device double) = E(Y) accumulated in FP64 from the
 * FP32 layout d_y [M][2], fixed-order reduction.  Asynchronous.             */
int ivhd_edges_stress(ivhd_edges *e, const float *d_y, float c, double *d_E);

/* ivhd_edges_grad: d_grad [M][2] = s * grad E(Y) in FP32, s = *d_scale (a
 * device float, e.g. the upstream gradient of a loss) or 1 when d_scale is
 * NULL.  Each vertex gathers its out- and in-edges in a fixed order (no
 * atomics; bitwise reproducible).  eps guards the rn unit vector.  Async.   */
int ivhd_edges_grad(ivhd_edges *e, const float *d_y, float c, float eps, const float *d_scale,
                    float *d_grad);

/* ivhd_edges_stress_grad: both of the above from one pass over the edges:
 * *d_E = E(Y) in FP64 (each out-edge's term as in ivhd_edges_stress, summed
 * per block of the gradient kernel and then in a fixed order, so equal to
 * ivhd_edges_stress up to summation order and bitwise reproducible) and
 * d_grad = s * grad E(Y) exactly as ivhd_edges_grad.  Same arguments and
 * errors as the two.  Asynchronous.                                         */
int ivhd_edges_stress_grad(ivhd_edges *e, const float *d_y, float c, float eps, const float *d_scale,
                           double *d_E, float *d_grad);

/* ivhd_scale_f32: d_out[k] = *d_scale * d_x[k] for k < n (device pointers,
 * d_out may equal d_x): the chain-rule step for a gradient taken before its
 * upstream scale was known.  n = 0 does nothing; n < 0 or a NULL pointer:
 * IVHD_EINVAL.  Asynchronous on `stream`.                                   */
int ivhd_scale_f32(const float *d_x, int64_t n, const float *d_scale, float *d_out, void *stream);

/* ivhd_edges_destroy: synchronises the plan's stream and frees it.         */
int ivhd_edges_destroy(ivhd_edges *e);

/* ivhd_grad_edges: one-shot gradient (plan created, used and destroyed):
 * d_grad = grad E(Y); if h_E is not NULL also *h_E = E(Y) (FP64).
 * Synchronises the stream.                                                 */
int ivhd_grad_edges(const float *d_y, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                    const int32_t *d_rn_idx, int32_t rn, float c, float eps, float *d_grad,
                    double *h_E, void *stream);

/* ivhd_grad_edges_noalloc: ivhd_grad_edges for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same kernels and the
 * same results bit for bit; it calls no hipMalloc or hipFree.  Its
 * temporaries (transposed lists, hub list, flags, FP64 stress partials)
 * live in one 64 MiB device array per GPU that the library holds until the
 * process ends.  Limit: about 4 (5 + nn + rn + max(nn, rn)) M bytes must
 * fit in 64 MiB (M up to about 1,670,000 at nn = 2, rn = 1, and 1,040,000
 * at nn = 5, rn = 1); larger inputs get IVHD_EINVAL before any device work.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (from other threads or streams) race.  Synchronises the stream.     */
int ivhd_grad_edges_noalloc(const float *d_y, int64_t M, const int32_t *d_nn_idx, int32_t nn,
                            const int32_t *d_rn_idx, int32_t rn, float c, float eps, float *d_grad,
                            double *h_E, void *stream);

/* ---- input preparation: exact kNN graph (brute force, FP32) ------------- */

/* ivhd_knn_build: the nn nearest neighbours of every row of X, the kNN graph
 * the loop embeds (its edges are the nn lists of Sec. "Improving classical
 * MDS"; the thesis obtains them from an approximate GPU index, this is the
 * exact graph).  Order: squared Euclidean distance, ties to the lower index,
 * the row itself excluded.
 *   d_x    float32 [M][N], row-major (read only)
 *   d_idx  int32 [M][k] output, nearest first
 * 1 <= k <= min(28, M-1), N >= 1.  Allocates a temporary [M] float buffer
 * and synchronises the stream.                                              */
int ivhd_knn_build(const float *d_x, int64_t M, int32_t N, int32_t k, int32_t *d_idx,
                   void *stream);

/* ---- approximate kNN: an inverted file over a k-means coarse quantizer ----
 * The thesis builds its kNN graphs with an approximate GPU library and
 * finds that graph construction dominates the end-to-end time (Sec.
 * "IVHD-CUDA").  This is the MI355X stand-in: points are grouped into nlist
 * lists by their nearest centroid; a query scans only the points of its
 * nprobe nearest lists (list-major: the queries probing a list are tiled
 * against the list's points on the matrix cores, as in ivhd_knn_build), and
 * the survivors are ranked by their exact FP32 distance.  nprobe = nlist - 1
 * or more lists makes it exact in practice; the recall at lower nprobe
 * depends on the data.                                                      */

/* ivhd_ivf_train: centroids started at the points floor(c M / nlist), then
 * n_iter Lloyd iterations (nearest centroid by squared distance, ties to
 * the lower index; each centroid moves to the FP32 mean of its points,
 * summed in id order; an empty list keeps its centroid), then the final
 * assignment.
 *   d_x          float32 [M][N] points (read only)
 *   d_centroids  float32 [nlist][N] output
 *   d_assign     int32 [M] output: the list of every point
 * 2 <= nlist <= M, n_iter >= 0.  Synchronises the stream.                   */
int ivhd_ivf_train(const float *d_x, int64_t M, int32_t N, int32_t nlist, int32_t n_iter,
                   float *d_centroids, int32_t *d_assign, void *stream);

/* ivhd_ivf_search: the k nearest points among the lists of the nprobe
 * centroids nearest to each query (order: exact FP32 squared distance,
 * ties to the lower index).
 *   d_x, M, N              the indexed points; d_centroids [nlist][N] and
 *                          d_assign [M] (entries in [0, nlist)) as from
 *                          ivhd_ivf_train (or any caller-made index)
 *   d_q [Q][N]             queries; d_self int32 [Q] or NULL: point
 *                          d_self[q] is excluded for query q (-1 = none)
 *   d_idx int32 [Q][k]     output (-1 where fewer than k points were probed);
 *   d_dist float32 [Q][k]  squared distances, or NULL
 * 1 <= k <= min(28, M-1), 1 <= nprobe <= min(28, nlist-1).  Allocates about
 * (4 (M + Q) N_pad + 8 Q nprobe k) bytes of temporaries and synchronises
 * the stream.                                                              */
int ivhd_ivf_search(const float *d_x, int64_t M, int32_t N, const float *d_centroids, int32_t nlist,
                    const int32_t *d_assign, const float *d_q, int64_t Q, const int32_t *d_self,
                    int32_t k, int32_t nprobe, int32_t *d_idx, float *d_dist, void *stream);

/* ivhd_rnn_mask: the reverse-neighbour pruning of Sec. "Reverse neighbors
 * mechanism".  An nn edge i -> j is kept when i is also among the kh
 * nearest neighbours of j in a wider helper graph (the thesis uses
 * kh = 4 nn), else its slot becomes -1; absent slots stay -1.  The result
 * is an nn list for a late-stage context.
 *   d_nn_idx  int32 [M][nn] (entries in [-1, M), no self edges)
 *   d_helper  int32 [M][kh], e.g. from ivhd_knn_build with k = kh
 *   d_out     int32 [M][nn]; may be d_nn_idx itself, not d_helper
 * 1 <= nn <= 64, 1 <= kh <= 256.  Synchronises the stream (validation).     */
int ivhd_rnn_mask(const int32_t *d_nn_idx, int64_t M, int32_t nn, const int32_t *d_helper, int32_t kh,
                  int32_t *d_out, void *stream);

/* ivhd_knn_query: the k nearest rows of X to each of Q query rows (used for
 * the quality metrics on a sample of points).
 *   d_q     float32 [Q][N] queries;  d_self int32 [Q] or NULL: row d_self[q]
 *           of X is excluded for query q (-1 = none)
 *   d_idx   int32 [Q][k];  d_dist float32 [Q][k] squared distances, or NULL
 * 1 <= k <= min(28, M-1).  Synchronises the stream.                         */
int ivhd_knn_query(const float *d_x, int64_t M, int32_t N, const float *d_q, int64_t Q,
                   const int32_t *d_self, int32_t k, int32_t *d_idx, float *d_dist,
                   void *stream);

/* ---- quality of a layout on a sample of points ---------------------------
 * The criteria of the thesis's chapter "Quality metrics", evaluated for a
 * sample of Q rows (d_rows, int32 [Q], entries in [0, M); the sample may be
 * every row).  The order of the points around a row r is all M points (r
 * included) by (delta_rl, l): delta the squared Euclidean distance summed in
 * FP64, dimension by dimension, from the FP32 coordinates; ties to the lower
 * index (the rank rho_rj of Sec. "Rank-based criteria").  Coordinates must
 * be finite.  These calls allocate temporaries and synchronise the stream. */

/* ivhd_eval_neighbours: d_idx int32 [Q][k] = the points at positions 1..k
 * of the order around each sample row (its neighbourhood of size k, Sec.
 * "Rank-based criteria"; position 0 is the row itself unless an identical
 * point of lower index precedes it).  d_z float32 [M][N], 1 <= N <= 1024,
 * 1 <= k <= min(128, M-1).                                                  */
int ivhd_eval_neighbours(const float *d_z, int64_t M, int32_t N, const int32_t *d_rows, int64_t Q,
                         int32_t k, int32_t *d_idx, void *stream);

/* ivhd_eval_ranks: d_rank int32 [Q][kc] = rho_rj for each sample row r and
 * each given point j = d_cand[q][c] (int32 [Q][kc], entries in [0, M)):
 * the number of points l with (delta_rl, l) before (delta_rj, j).
 * 1 <= kc <= 64.                                                            */
int ivhd_eval_ranks(const float *d_z, int64_t M, int32_t N, const int32_t *d_rows, int64_t Q,
                    const int32_t *d_cand, int32_t kc, int32_t *d_rank, void *stream);

/* ivhd_eval_scores: the sample criteria at size k from neighbour lists in
 * the data (d_nx [Q][kx], may be NULL) and in the layout (d_ny [Q][ky]),
 * both as from ivhd_eval_neighbours:
 *   h_out[0] = Q_NX(k) = sum_q |v_q ∩ n_q| / (k Q)   (Sec. "Rank-based
 *              criteria"; NaN when d_nx is NULL)
 *   h_out[1] = cf_k = share of the layout neighbours carrying the row's
 *              label (Sec. "Neighbor hit"; d_labels int32 [M]; NaN when NULL)
 *   h_out[2] = T(k) = 1 - 2 / (Q k (2M - 3k - 1)) sum_q sum_{j in n_q \ v_q}
 *              (rho^X_{r_q j} - k)   (trustworthiness, Sec. "Trustworthiness
 *              and continuity", over the sample; d_rank_y [Q][ky] = the data
 *              ranks of the layout neighbours, as from ivhd_eval_ranks; NaN
 *              when NULL).  With every row as the sample these are the
 *              criteria of the whole layout.
 * 1 <= k <= ky (and <= kx when d_nx is given), Q >= 1.                      */
int ivhd_eval_scores(int64_t M, const int32_t *d_rows, int64_t Q, const int32_t *d_nx, int32_t kx,
                     const int32_t *d_ny, int32_t ky, const int32_t *d_rank_y, const int32_t *d_labels,
                     int32_t k, double *h_out, void *stream);

/* ---- parametric encoder --------------------------------------------------
 * A learned map N-D -> 2-D: MLP n_in -> h1 -> h2 -> 2 with ReLU, trained on
 * the IVHD stress of its own batches' edges, so that new points are placed
 * in one forward pass.  (Not in the thesis; its MLP conventions follow the
 * network-inspection chapter: ReLU layers, Glorot-uniform initialisation.)
 * BF16 weights and activations on the matrix cores with FP32 accumulation;
 * FP32 master weights and Adam state (beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8, bias correction 1/(1 - beta^t)).  Every FP32 -> BF16
 * conversion rounds to nearest even; ReLU is applied in FP32 before it; the
 * output Z stays FP32.
 * Parameter layout (FP32, flat): W1 [h1][n_in], b1 [h1], W2 [h2][h1],
 * b2 [h2], W3 [2][h2], b3 [2].                                             */
typedef struct ivhd_enc ivhd_enc;   /* opaque */

/* ivhd_enc_create: Glorot-uniform weights (s = sqrt(6/(fan_in+fan_out)))
 * from `seed`, zero biases.  h1, h2 multiples of 8.  max_rows bounds the
 * rows of one forward/training call (activation buffers are sized for it).
 * Synchronises the stream.                                                 */
int ivhd_enc_create(ivhd_enc **out, int32_t n_in, int32_t h1, int32_t h2, uint64_t seed,
                    int64_t max_rows, void *stream);
int ivhd_enc_num_params(const ivhd_enc *e, int64_t *h_n);
/* copy the FP32 parameters and/or the last step's (unscaled) gradients into
 * device buffers of ivhd_enc_num_params floats (either may be NULL).       */
int ivhd_enc_get_params(ivhd_enc *e, float *d_params, float *d_grads);
/* load FP32 parameters (device); resets the Adam state.                    */
int ivhd_enc_set_params(ivhd_enc *e, const float *d_params);

/* ivhd_enc_embed: d_z float32 [rows][2] = the network applied to d_x16
 * (BF16 [rows][n_in], row-major).  Asynchronous.                           */
int ivhd_enc_embed(ivhd_enc *e, const uint16_t *d_x16, int64_t rows, float *d_z);

/* ivhd_enc_train_step: one Adam step on a batch of R rows (BF16
 * [R][n_in]) whose local edge lists are the plan's (indices into the R
 * rows): loss = loss_scale * E_batch(Z); gradients of E_batch are scaled
 * by loss_scale before Adam.  *d_loss (device double, may be NULL) gets
 * E_batch.  Asynchronous.                                                  */
int ivhd_enc_train_step(ivhd_enc *e, const uint16_t *d_xb16, int64_t R, ivhd_edges *plan, float c,
                        float eps, float lr, float loss_scale, double *d_loss);

/* ivhd_enc_train_epoch: one pass over M training points (BF16 [M][n_in])
 * in batches of `batch` sources visited in the order (a b + c0) mod M
 * (gcd(a, M) = 1, both drawn from seed and epoch).  A batch forwards its
 * sources, their nn targets (d_nn_idx [M][nn]; an absent slot repeats the
 * source) and their rn targets (drawn for this epoch exactly as the loop
 * draws epoch `epoch`), and takes one Adam step on the mean per-source
 * stress of those edges.  batch * (1 + nn + rn) <= max_rows.  *h_loss =
 * mean over steps of that loss.  Synchronises the stream.                  */
int ivhd_enc_train_epoch(ivhd_enc *e, const uint16_t *d_x16, int64_t M, const int32_t *d_nn_idx,
                         int32_t nn, int32_t rn, uint64_t seed, int64_t epoch, int64_t batch,
                         float c, float eps, float lr, double *h_loss);
int ivhd_enc_destroy(ivhd_enc *e);

/* ivhd_f32_to_bf16: d_y[i] = round-to-nearest-even BF16 of d_x[i].  Async. */
int ivhd_f32_to_bf16(const float *d_x, int64_t n, uint16_t *d_y, void *stream);

/* ivhd_gemm_bf16: C[M][N] = sum_k opA[m][k] opB[k][n] on the matrix cores,
 * BF16 operands, FP32 accumulation.
 *   opA[m][k] = trans_a ? A[k*lda + m] : A[m*lda + k]
 *   opB[k][n] = trans_b ? B[n*ldb + k] : B[k*ldb + n]
 * epilogue 0: C FP32;  1: C BF16 = relu(acc + bias[n]) (bias may be NULL);
 *          2: C BF16 = acc if mask[m*ldm + n] > 0 else 0 (ReLU derivative).
 * splits > 1 splits K (epilogue 0 only): FP32 partials go to d_work
 * [splits][M][N] and are added in split order into C.  Asynchronous.      */
int ivhd_gemm_bf16(const uint16_t *d_a, const uint16_t *d_b, int64_t M, int64_t N, int64_t K,
                   int64_t lda, int64_t ldb, int32_t trans_a, int32_t trans_b, int32_t epilogue,
                   const float *d_bias, const uint16_t *d_mask, int64_t ldm, void *d_c, int64_t ldc,
                   int32_t splits, float *d_work, void *stream);

/* ivhd_last_error: message of the last failure on this thread ("" if none). */
const char *ivhd_last_error(void);

/* ivhd_version: library version as major*10000 + minor*100 + patch.        */
int ivhd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IVHD_H */
