/*
 * Plain FP64 CPU oracle of the IVHD embedding loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it shares no code, header or constant table with the
 * HIP path.  Its only callers are the tests, the smoke check and the CPU
 * baseline leg of the benchmark.
 *
 * Every function is the definition written out, one edge at a time, in the
 * order the thesis states it, with no blocking, fusion or reordering:
 *
 *   stress   E(Y) = sum_i [ sum_{j in O_nn(i)} d_ij^2
 *                           + c * sum_{k in O_rn(i)} (1 - d_ik)^2 ]
 *            (Sec. "Improving classical MDS", Eq. ivhd_cost_function;
 *             binary targets 0 / 1 of Eq. ivhd_binary_distances)
 *   force    f = -1/2 grad E, assembled edge by edge, each directed edge
 *            acting on both of its ends with opposite signs (IVHD-CUDA
 *            section: one positive and one negative slot per connection).
 *            nn edge (i,j): F = -(y_i - y_j)                       (Eq. eq13)
 *            rn edge (i,k): F = +c (1 - d) (y_i - y_k) / max(d, eps)
 *            The sign of the rn term follows -1/2 grad of the stress; the
 *            printed Eq. eq13 carries the opposite sign (a misprint: with
 *            it the random edges would pull points together).
 *   step     V <- a V + b f ;  Y <- Y + V, all vertices from the same Y_n
 *            (Eq. ivhd_force_1 / ivhd_position_update; Eq.
 *             force_directed_update of Sec. "Force directed").
 *            Nesterov variant (Sec. "Optimization methods", Nesterov): the
 *            force is taken at the look-ahead layout Y + a V.
 *   metric   d is the Euclidean distance; the late-stage variant of Sec.
 *            "L1 norm in late stages of embedding" uses d = |dx| + |dy| in
 *            the same stress, and its force is again -1/2 grad E, with the
 *            subgradient sign(0) = 0 where a coordinate difference vanishes:
 *            nn edge: F = -d (sign dx, sign dy)
 *            rn edge: F = +c (1 - d) (sign dx, sign dy)
 *   adapt    self-adaptive b of Sec. "Force directed": each step is first
 *            taken tentatively; with dT = sum_i |V'_i|^2 - |V_i|^2 (the change
 *            of kinetic energy), |dT| > tau rejects the step (Y and V stay)
 *            and scales b by g1 > 1 when dT < -tau or by g2 < 1 when
 *            dT > tau (or dT is not finite); otherwise the step is kept and
 *            b stays.
 *   adam     Adam of Sec. "Optimization methods" on g = grad E = -2 f, per
 *            coordinate: m <- b1 m + (1 - b1) g, s <- b2 s + (1 - b2) g^2,
 *            Y <- Y - lr (m / (1 - b1^t)) / (eps + sqrt(s / (1 - b2^t))),
 *            t = 1, 2, ... the Adam step count (textbook bias correction).
 *   mask     reverse-neighbour pruning of Sec. "Reverse neighbors
 *            mechanism": an nn edge i -> j is kept only when i is also
 *            among the kh nearest neighbours of j in a wider helper graph.
 *   rn       per vertex, rn distinct random non-neighbours other than
 *            itself, drawn ad hoc (Sec. "Improving classical MDS"; the
 *            practical rules of Sec. "Force directed": a connected
 *            neighbour cannot be a random one).  The draws come from the
 *            counter-based SplitMix64 generator (Steele, Lea and Flood,
 *            OOPSLA 2014; Vigna's public-domain reference), keyed by
 *            (seed, epoch, vertex, slot, try).
 *
 * Threaded loop (orc_run_threads): the same iterations with the force of
 * each step gathered per vertex by OpenMP threads.  Vertex v adds the terms
 * of its incident edges in the order of the edge list above (source row,
 * then slot), which is exactly the order in which orc_force adds them to
 * f[v]; each term is computed from the same operands in the same order, so
 * the result equals orc_run bit for bit for any thread count.  It exists
 * only to time the oracle on every host core.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

/* ---- SplitMix64: state advanced by the golden gamma, then the mix ---- */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Random-neighbour draw for one epoch.
 * For vertex i and slot r the t-th try is
 *     ctr = ((epoch * M + i) * rn + r) * 256 + t
 *     h   = splitmix64(seed XOR splitmix64(ctr))
 *     j   = h mod (M - 1), shifted past i (so j != i, uniform on the rest)
 * A try is rejected when j is an nn out-neighbour of i or was already drawn
 * for i; the try with t = 255 is accepted whatever it gives.            */
static void rn_sample_rows(int64_t M, int32_t nn, const int32_t *nn_idx, int32_t rn,
                           uint64_t seed, int64_t epoch, int32_t *rn_out, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        for (int32_t r = 0; r < rn; ++r) {
            int64_t pick = -1;
            for (int t = 0; t < 256; ++t) {
                uint64_t ctr = (((uint64_t)epoch * (uint64_t)M + (uint64_t)i) * (uint64_t)rn
                                + (uint64_t)r) * 256u + (uint64_t)t;
                uint64_t h = orc_splitmix64(seed ^ orc_splitmix64(ctr));
                int64_t j = (int64_t)(h % (uint64_t)(M - 1));
                if (j >= i) j += 1;
                int clash = 0;
                for (int32_t q = 0; q < nn; ++q)
                    if (nn_idx[i * nn + q] == j) clash = 1;
                for (int32_t q = 0; q < r; ++q)
                    if (rn_out[i * rn + q] == j) clash = 1;
                pick = j;
                if (!clash) break;
            }
            rn_out[i * rn + r] = (int32_t)pick;
        }
    }
}

void orc_rn_sample(int64_t M, int32_t nn, const int32_t *nn_idx, int32_t rn,
                   uint64_t seed, int64_t epoch, int32_t *rn_out)
{
    rn_sample_rows(M, nn, nn_idx, rn, seed, epoch, rn_out, 0, M);
}

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

/* f = -1/2 grad E, edge by edge; f must hold 2*M doubles (overwritten).
 * metric 0: Euclidean distance, 1: l1 distance.                        */
void orc_force(int64_t M, const double *Y, int32_t nn, const int32_t *nn_idx,
               int32_t rn, const int32_t *rn_idx, double c, double eps, int32_t metric,
               double *f)
{
    for (int64_t i = 0; i < 2 * M; ++i) f[i] = 0.0;
    for (int64_t i = 0; i < M; ++i) {
        for (int32_t q = 0; q < nn; ++q) {
            int64_t j = nn_idx[i * nn + q];
            if (j < 0) continue;                      /* absent neighbour */
            double dx = Y[2 * i] - Y[2 * j];
            double dy = Y[2 * i + 1] - Y[2 * j + 1];
            double Fx, Fy;
            if (metric == 0) {                        /* -1/2 d/dy_i of d^2 */
                Fx = -dx;
                Fy = -dy;
            } else {
                double d = fabs(dx) + fabs(dy);
                Fx = -d * sgn(dx);
                Fy = -d * sgn(dy);
            }
            f[2 * i] += Fx;  f[2 * i + 1] += Fy;
            f[2 * j] -= Fx;  f[2 * j + 1] -= Fy;
        }
        for (int32_t q = 0; q < rn; ++q) {
            int64_t k = rn_idx[i * rn + q];
            if (k < 0) continue;                      /* absent slot */
            double dx = Y[2 * i] - Y[2 * k];
            double dy = Y[2 * i + 1] - Y[2 * k + 1];
            double Fx, Fy;
            if (metric == 0) {                        /* -1/2 d/dy_i of c (1 - d)^2 */
                double d = sqrt(dx * dx + dy * dy);
                double s = c * (1.0 - d) / (d > eps ? d : eps);
                Fx = s * dx;
                Fy = s * dy;
            } else {
                double d = fabs(dx) + fabs(dy);
                Fx = c * (1.0 - d) * sgn(dx);
                Fy = c * (1.0 - d) * sgn(dy);
            }
            f[2 * i] += Fx;  f[2 * i + 1] += Fy;
            f[2 * k] -= Fx;  f[2 * k + 1] -= Fy;
        }
    }
}

double orc_stress(int64_t M, const double *Y, int32_t nn, const int32_t *nn_idx,
                  int32_t rn, const int32_t *rn_idx, double c, int32_t metric)
{
    double E = 0.0;
    for (int64_t i = 0; i < M; ++i) {
        for (int32_t q = 0; q < nn; ++q) {
            int64_t j = nn_idx[i * nn + q];
            if (j < 0) continue;
            double dx = Y[2 * i] - Y[2 * j];
            double dy = Y[2 * i + 1] - Y[2 * j + 1];
            double d = metric == 0 ? sqrt(dx * dx + dy * dy) : fabs(dx) + fabs(dy);
            E += metric == 0 ? dx * dx + dy * dy : d * d;   /* d_ij^2 */
        }
        for (int32_t q = 0; q < rn; ++q) {
            int64_t k = rn_idx[i * rn + q];
            if (k < 0) continue;
            double dx = Y[2 * i] - Y[2 * k];
            double dy = Y[2 * i + 1] - Y[2 * k + 1];
            double d = metric == 0 ? sqrt(dx * dx + dy * dy) : fabs(dx) + fabs(dy);
            E += c * (1.0 - d) * (1.0 - d);           /* c (1 - d_ik)^2 */
        }
    }
    return E;
}

/* Reverse-neighbour mask: out[i][q] = nn_idx[i][q] when that j >= 0 lists
 * i among its first kh helper neighbours, else -1.                      */
void orc_rnn_mask(int64_t M, int32_t nn, const int32_t *nn_idx, int32_t kh,
                  const int32_t *helper, int32_t *out)
{
    for (int64_t i = 0; i < M; ++i) {
        for (int32_t q = 0; q < nn; ++q) {
            int64_t j = nn_idx[i * nn + q];
            int keep = 0;
            if (j >= 0)
                for (int32_t r = 0; r < kh; ++r)
                    if (helper[j * kh + r] == i) keep = 1;
            out[i * nn + q] = keep ? (int32_t)j : -1;
        }
    }
}

/* T iterations starting at iteration n0.  Y, V: 2*M doubles, updated in
 * place.  rn_idx: M*rn ints, in/out.  f, Yh: 2*M doubles of scratch.
 * The random neighbours of epoch e = (R > 0 ? n / R : 0) are drawn at the
 * first iteration of the call and whenever n is a multiple of R.
 * nesterov != 0: the force of each step is taken at Yh = Y + a V.       */
void orc_run(int64_t M, double *Y, double *V, int32_t nn, const int32_t *nn_idx,
             int32_t rn, int32_t *rn_idx, double a, double b, double c, double eps,
             uint64_t seed, int64_t R, int64_t n0, int64_t T, int32_t nesterov,
             int32_t metric, double *f, double *Yh)
{
    for (int64_t n = n0; n < n0 + T; ++n) {
        if (n == n0 || (R > 0 && n % R == 0))
            orc_rn_sample(M, nn, nn_idx, rn, seed, R > 0 ? n / R : 0, rn_idx);
        if (nesterov) {
            for (int64_t i = 0; i < 2 * M; ++i) Yh[i] = Y[i] + a * V[i];
            orc_force(M, Yh, nn, nn_idx, rn, rn_idx, c, eps, metric, f);
        } else {
            orc_force(M, Y, nn, nn_idx, rn, rn_idx, c, eps, metric, f);
        }
        for (int64_t i = 0; i < 2 * M; ++i) {
            V[i] = a * V[i] + b * f[i];
            Y[i] = Y[i] + V[i];
        }
    }
}

/* T iterations of the plain loop with the self-adaptive b, from iteration
 * n0.  *b is read and updated.  Per step k (0-based) it records the kinetic
 * energy change dT[k], the b used bs[k] and acc[k] = 1 (kept) or 0
 * (rejected); any of them may be NULL.  Vt, Yt, f: 2*M doubles of scratch.
 * Returns the number of kept steps.                                      */
int64_t orc_run_adaptive(int64_t M, double *Y, double *V, int32_t nn, const int32_t *nn_idx,
                         int32_t rn, int32_t *rn_idx, double a, double *b, double c,
                         double eps, uint64_t seed, int64_t R, int64_t n0, int64_t T,
                         double tau, double g1, double g2, int32_t metric, double *dT,
                         double *bs, int32_t *acc, double *f, double *Yt, double *Vt)
{
    int64_t kept = 0;
    for (int64_t n = n0; n < n0 + T; ++n) {
        if (n == n0 || (R > 0 && n % R == 0))
            orc_rn_sample(M, nn, nn_idx, rn, seed, R > 0 ? n / R : 0, rn_idx);
        orc_force(M, Y, nn, nn_idx, rn, rn_idx, c, eps, metric, f);
        double d = 0.0;
        for (int64_t i = 0; i < M; ++i) {
            double vx = a * V[2 * i] + *b * f[2 * i];
            double vy = a * V[2 * i + 1] + *b * f[2 * i + 1];
            Vt[2 * i] = vx;
            Vt[2 * i + 1] = vy;
            Yt[2 * i] = Y[2 * i] + vx;
            Yt[2 * i + 1] = Y[2 * i + 1] + vy;
            d += (vx * vx + vy * vy) - (V[2 * i] * V[2 * i] + V[2 * i + 1] * V[2 * i + 1]);
        }
        int64_t k = n - n0;
        if (bs) bs[k] = *b;
        if (dT) dT[k] = d;
        int keep = isfinite(d) && fabs(d) <= tau;   /* a non-finite dT counts as a rise */
        if (keep) {
            for (int64_t i = 0; i < 2 * M; ++i) {
                Y[i] = Yt[i];
                V[i] = Vt[i];
            }
            ++kept;
        } else {
            *b *= d < -tau ? g1 : g2;
        }
        if (acc) acc[k] = keep;
    }
    return kept;
}

/* T Adam iterations from iteration n0; t0 Adam steps were taken before (the
 * first step here uses t = t0 + 1).  Y, Mo (first moment), S (second
 * moment): 2*M doubles, updated in place.  f: 2*M doubles of scratch.     */
void orc_run_adam(int64_t M, double *Y, double *Mo, double *S, int32_t nn, const int32_t *nn_idx,
                  int32_t rn, int32_t *rn_idx, double lr, double b1, double b2, double eps_a,
                  double c, double eps, uint64_t seed, int64_t R, int64_t n0, int64_t T,
                  int64_t t0, int32_t metric, double *f)
{
    for (int64_t n = n0; n < n0 + T; ++n) {
        if (n == n0 || (R > 0 && n % R == 0))
            orc_rn_sample(M, nn, nn_idx, rn, seed, R > 0 ? n / R : 0, rn_idx);
        orc_force(M, Y, nn, nn_idx, rn, rn_idx, c, eps, metric, f);
        double t = (double)(t0 + (n - n0) + 1);
        double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
        for (int64_t i = 0; i < 2 * M; ++i) {
            double g = -2.0 * f[i];
            Mo[i] = b1 * Mo[i] + (1.0 - b1) * g;
            S[i] = b2 * S[i] + (1.0 - b2) * g * g;
            Y[i] = Y[i] - lr * (Mo[i] / c1) / (eps_a + sqrt(S[i] / c2));
        }
    }
}

/* Incidence lists of the edges of one draw: for every vertex v, the ids of
 * the edges that touch it, ascending.  Edge id = row * (nn + rn) + slot,
 * slots 0..nn-1 for nn, nn..nn+rn-1 for rn; absent slots are left out.
 * ptr: M + 1 entries, ids: 2 * M * (nn + rn) entries.                    */
static void incidence(int64_t M, int32_t nn, const int32_t *nn_idx, int32_t rn,
                      const int32_t *rn_idx, int64_t *ptr, int64_t *ids)
{
    const int64_t w = nn + rn;
    for (int64_t v = 0; v <= M; ++v) ptr[v] = 0;
    for (int64_t i = 0; i < M; ++i)
        for (int32_t q = 0; q < w; ++q) {
            int64_t o = q < nn ? nn_idx[i * nn + q] : rn_idx[i * rn + (q - nn)];
            if (o < 0) continue;
            ptr[i + 1] += 1;
            ptr[o + 1] += 1;
        }
    for (int64_t v = 0; v < M; ++v) ptr[v + 1] += ptr[v];
    int64_t *fill = (int64_t *)malloc((size_t)M * sizeof(int64_t));
    for (int64_t v = 0; v < M; ++v) fill[v] = ptr[v];
    /* edges visited in id order, so every list ends up ascending */
    for (int64_t i = 0; i < M; ++i)
        for (int32_t q = 0; q < w; ++q) {
            int64_t o = q < nn ? nn_idx[i * nn + q] : rn_idx[i * rn + (q - nn)];
            if (o < 0) continue;
            ids[fill[i]++] = i * w + q;
            ids[fill[o]++] = i * w + q;
        }
    free(fill);
}

/* f = -1/2 grad E by a per-vertex gather over the incidence lists: the
 * term F of edge (i, o) is computed as in orc_force and added at i,
 * subtracted at o.                                                        */
static void force_gather(int64_t M, const double *Y, int32_t nn, const int32_t *nn_idx,
                         int32_t rn, const int32_t *rn_idx, double c, double eps,
                         int32_t metric, const int64_t *ptr, const int64_t *ids, double *f)
{
    const int64_t w = nn + rn;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < M; ++v) {
        double fx = 0.0, fy = 0.0;
        for (int64_t p = ptr[v]; p < ptr[v + 1]; ++p) {
            const int64_t e = ids[p], i = e / w;
            const int32_t q = (int32_t)(e % w);
            const int rnd = q >= nn;
            const int64_t o = rnd ? rn_idx[i * rn + (q - nn)] : nn_idx[i * nn + q];
            double dx = Y[2 * i] - Y[2 * o];
            double dy = Y[2 * i + 1] - Y[2 * o + 1];
            double Fx, Fy;
            if (!rnd) {
                if (metric == 0) {
                    Fx = -dx;
                    Fy = -dy;
                } else {
                    double d = fabs(dx) + fabs(dy);
                    Fx = -d * sgn(dx);
                    Fy = -d * sgn(dy);
                }
            } else if (metric == 0) {
                double d = sqrt(dx * dx + dy * dy);
                double s = c * (1.0 - d) / (d > eps ? d : eps);
                Fx = s * dx;
                Fy = s * dy;
            } else {
                double d = fabs(dx) + fabs(dy);
                Fx = c * (1.0 - d) * sgn(dx);
                Fy = c * (1.0 - d) * sgn(dy);
            }
            if (i == v) {
                fx += Fx;
                fy += Fy;
            } else {
                fx -= Fx;
                fy -= Fy;
            }
        }
        f[2 * v] = fx;
        f[2 * v + 1] = fy;
    }
}

/* orc_run on nthreads OpenMP threads (same arguments, same result). */
void orc_run_threads(int64_t M, double *Y, double *V, int32_t nn, const int32_t *nn_idx,
                     int32_t rn, int32_t *rn_idx, double a, double b, double c, double eps,
                     uint64_t seed, int64_t R, int64_t n0, int64_t T, int32_t nesterov,
                     int32_t metric, double *f, double *Yh, int32_t nthreads)
{
    const int64_t cap = 2 * M * (int64_t)(nn + rn);
    int64_t *ptr = (int64_t *)malloc((size_t)(M + 1) * sizeof(int64_t));
    int64_t *ids = (int64_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int64_t));
    omp_set_num_threads(nthreads > 0 ? nthreads : 1);
    for (int64_t n = n0; n < n0 + T; ++n) {
        if (n == n0 || (R > 0 && n % R == 0)) {
            /* every vertex's draw is a function of (seed, epoch, vertex) alone */
            const int64_t chunk = 4096;
#pragma omp parallel for schedule(static)
            for (int64_t i0 = 0; i0 < M; i0 += chunk)
                rn_sample_rows(M, nn, nn_idx, rn, seed, R > 0 ? n / R : 0, rn_idx, i0,
                               i0 + chunk < M ? i0 + chunk : M);
            incidence(M, nn, nn_idx, rn, rn_idx, ptr, ids);
        }
        const double *Yf = Y;
        if (nesterov) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < 2 * M; ++i) Yh[i] = Y[i] + a * V[i];
            Yf = Yh;
        }
        force_gather(M, Yf, nn, nn_idx, rn, rn_idx, c, eps, metric, ptr, ids, f);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < 2 * M; ++i) {
            V[i] = a * V[i] + b * f[i];
            Y[i] = Y[i] + V[i];
        }
    }
    free(ptr);
    free(ids);
}
