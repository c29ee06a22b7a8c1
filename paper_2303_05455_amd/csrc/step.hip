// One IVHD iteration on gfx950 (Sec. "Force directed", Eq.
// force_directed_update, with the force of Eq. eq13 taken as -1/2 grad of
// Eq. ivhd_cost_function):
//
//   every edge incident to vertex i, whichever way it points, acts on i with
//     nn edge:  -(y_i - y_o)
//     rn edge:  c (1 - d) (y_i - y_o) / max(d, eps),   d = |y_i - y_o|
//   f_i = sum of those;   v_i <- a v_i + b f_i ;   y_i <- y_i + v_i
//
// Deterministic mode.  Each vertex gathers its out-edges (rows of nn_idx /
// rn_idx) and its in-edges (the transposed lists, sources ascending) and
// then updates v in place and writes y to the other half of a ping-pong
// pair, so no thread reads a position another thread has already moved.
// Force and update are fused: one kernel per iteration, no force array.
//
// kNN graphs of high-dimensional data have hubs (in-degrees of hundreds at
// 1.4M points), and a hub walked by one thread serialises the whole
// iteration behind its chain of dependent loads.  So the work is split by
// degree:
//   * the first `heavy_blocks` blocks give each vertex of nn in-degree above
//     heavy_deg a whole wavefront: the 64 lanes stride over its edge list
//     and a fixed xor-butterfly adds their partial sums;
//   * the other blocks give each remaining vertex one thread, which issues
//     its in-edge gathers eight (then four) at a time so several loads are
//     in flight -- or, on graphs too small to fill the chip that way, a
//     group of four lanes that share its edge list like a hub's wavefront.
// Both orders of summation are fixed, so results are bitwise reproducible.
//
// Atomic mode: pass 1 is the deterministic kernel's walk without the rn
// in-edges: each vertex gathers its nn edges both ways and its rn out-edges
// (its own share, stored to fown) and adds each rn out-edge's reaction to
// the other end's accumulator with atomics; pass 2 adds them up, applies the
// update and clears the accumulators.  Atomics run at a fixed rate per
// operation on this chip whatever the footprint or memory scope (measured:
// about 21 G/s for 32-bit float adds, 23 G/s for 64-bit integer adds), so
// the mode keeps them to the rn edges and gives each reaction one 64-bit
// integer atomic: x and y in fixed point, packed.  Integer sums do not
// depend on the order of arrival, so the mode is bitwise reproducible as
// long as every reaction fits the fixed-point range (the rare ones that do
// not take two float atomics).
//
// Variants of the thesis, chosen per context and compiled as template
// parameters so the plain loop carries none of their cost:
//   L1     the distance is |dx| + |dy| (Sec. "L1 norm in late stages of
//          embedding"); the force is again -1/2 grad E, with sign(0) = 0:
//            nn edge: -d (sign dx, sign dy);  rn edge: c (1 - d) (sign dx, sign dy)
//   NEST   Nesterov look-ahead (Sec. "Optimization methods"): forces are
//          gathered from H = Y + a V, which each update also writes for the
//          next iteration (one more position array, no extra gathers)
//   ADAPT  the self-adaptive b of Sec. "Force directed": the step is
//          tentative (V is written to a second buffer), b is read from
//          device memory, and each block leaves the FP64 sum of
//          |v'|^2 - |v|^2 over its vertices for the accept / reject decision.
//   ADAM   Adam (Sec. "Optimization methods") on g = grad E = -2 f per
//          coordinate; V holds the first moments, a second array the second
//          moments, and the bias corrections of the step come from device
//          memory (one tiny kernel per iteration advances them).
// (NEST, ADAPT and ADAM are the values of one template argument, OPT.)
#include "ivhd_internal.h"

namespace ivhd {
namespace {

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

template <bool L1>
__device__ __forceinline__ float2 nn_term(float2 yi, float2 yo) {
  if (L1) {
    const float dx = yi.x - yo.x, dy = yi.y - yo.y;
    const float d = fabsf(dx) + fabsf(dy);
    return make_float2(-d * sgnf(dx), -d * sgnf(dy));
  }
  return make_float2(yo.x - yi.x, yo.y - yi.y);
}

template <bool L1>
__device__ __forceinline__ float2 rn_term(float2 yi, float2 yo, float c, float eps) {
  const float dx = yi.x - yo.x, dy = yi.y - yo.y;
  if (L1) {
    const float s = c * (1.0f - (fabsf(dx) + fabsf(dy)));
    return make_float2(s * sgnf(dx), s * sgnf(dy));
  }
  const float d = sqrtf(dx * dx + dy * dy);
  const float s = c * (1.0f - d) / fmaxf(d, eps);
  return make_float2(s * dx, s * dy);
}

// an out-edge's share of Eq. ivhd_cost_function in FP64, from the FP32
// positions widened before subtracting (the terms of the stress kernel)
template <bool L1>
__device__ __forceinline__ double nn_stress(float2 yi, float2 yo) {
  const double dx = (double)yi.x - (double)yo.x, dy = (double)yi.y - (double)yo.y;
  if (L1) {
    const double d = fabs(dx) + fabs(dy);
    return d * d;
  }
  return dx * dx + dy * dy;
}

template <bool L1>
__device__ __forceinline__ double rn_stress(float2 yi, float2 yo, double c) {
  const double dx = (double)yi.x - (double)yo.x, dy = (double)yi.y - (double)yo.y;
  const double d = L1 ? fabs(dx) + fabs(dy) : sqrt(dx * dx + dy * dy);
  return c * (1.0 - d) * (1.0 - d);
}

// atomic mode: the reaction -t of an rn out-edge on its other end k.  Both
// coordinates in units of A.rx_unit, rounded to the nearest integer, go to
// k's fixed-point accumulator in one 64-bit integer atomic (y in the high
// field, x in the low one, as y 2^32 + x); a reaction outside the range of
// the current draw (or not finite) goes to the float accumulator instead.
__device__ __forceinline__ void add_reaction(const StepArgs &A, int32_t k, float2 t) {
  const float cap = A.rx->cap;
  const float qx = -t.x * A.rx_inv_unit, qy = -t.y * A.rx_inv_unit;
  if (fabsf(qx) <= cap && fabsf(qy) <= cap) {
    const int32_t ix = (int32_t)rintf(qx), iy = (int32_t)rintf(qy);
    const uint64_t w = ((uint64_t)(uint32_t)iy << 32) + (uint64_t)(int64_t)ix;
    atomicAdd((unsigned long long *)&A.facc[k], (unsigned long long)w);
  } else {
    unsafeAtomicAdd(&A.fbuf[k].x, -t.x);
    unsafeAtomicAdd(&A.fbuf[k].y, -t.y);
    A.fflag[A.fpar] = 1;
  }
}

// the two fields of a fixed-point accumulator, in float
__device__ __forceinline__ float2 fixed_reactions(uint64_t w, float unit) {
  const int32_t x = (int32_t)(uint32_t)w;
  const int32_t y = (int32_t)(uint32_t)((w - (uint64_t)(int64_t)x) >> 32);
  return make_float2((float)x * unit, (float)y * unit);
}

// in-edge segment [s, e) of a light vertex, eight (then four) gathers in
// flight at a time; the terms are still added one by one in ascending order
template <bool RN, bool L1>
__device__ __forceinline__ void gather_segment(const float2 *__restrict__ y, const int32_t *__restrict__ src,
                                               int32_t s, int32_t e, float2 yi, float c, float eps,
                                               float &fx, float &fy) {
  int32_t p = s;
  for (; p + 8 <= e; p += 8) {
    int32_t j[8];
    float2 yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) j[u] = src[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) yv[u] = y[j[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float2 t = RN ? rn_term<L1>(yi, yv[u], c, eps) : nn_term<L1>(yi, yv[u]);
      fx += t.x; fy += t.y;
    }
  }
  for (; p + 4 <= e; p += 4) {
    const int32_t j0 = src[p], j1 = src[p + 1], j2 = src[p + 2], j3 = src[p + 3];
    const float2 y0 = y[j0], y1 = y[j1], y2 = y[j2], y3 = y[j3];
    float2 t;
    t = RN ? rn_term<L1>(yi, y0, c, eps) : nn_term<L1>(yi, y0); fx += t.x; fy += t.y;
    t = RN ? rn_term<L1>(yi, y1, c, eps) : nn_term<L1>(yi, y1); fx += t.x; fy += t.y;
    t = RN ? rn_term<L1>(yi, y2, c, eps) : nn_term<L1>(yi, y2); fx += t.x; fy += t.y;
    t = RN ? rn_term<L1>(yi, y3, c, eps) : nn_term<L1>(yi, y3); fx += t.x; fy += t.y;
  }
  for (; p < e; ++p) {
    const float2 t = RN ? rn_term<L1>(yi, y[src[p]], c, eps) : nn_term<L1>(yi, y[src[p]]);
    fx += t.x; fy += t.y;
  }
}

// force on a light vertex: out-nn, out-rn, in-nn, in-rn, in that order.
// Positions are gathered from A.h (Y, or the look-ahead H = Y + a V).
// With ARN (atomic mode) the rn in-edges are not gathered: each rn
// out-edge's reaction goes to the other end's accumulator by add_reaction.
// With ST the out-edges' stress terms are added to es in FP64 (out-nn, then
// out-rn).
template <bool L1, bool ARN, bool ST = false>
__device__ __forceinline__ float2 light_force(const StepArgs &A, int64_t i, float2 yi, int32_t ns,
                                              int32_t ne, double &es) {
  const float2 *__restrict__ y = A.h;
  float fx = 0.f, fy = 0.f;
  const int32_t *__restrict__ out_nn = A.nn_idx + i * A.nn;
  int q = 0;
  // four out-nn edges at a time (their loads in flight together; an absent
  // slot reads the vertex itself and adds nothing), terms in edge order
  for (; q + 4 <= A.nn; q += 4) {
    int32_t j[4];
    float2 yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) j[u] = out_nn[q + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) yv[u] = y[j[u] >= 0 ? (int64_t)j[u] : i];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j[u] < 0) continue;
      const float2 t = nn_term<L1>(yi, yv[u]);
      fx += t.x; fy += t.y;
      if (ST) es += nn_stress<L1>(yi, yv[u]);
    }
  }
  for (; q < A.nn; ++q) {
    const int32_t j = out_nn[q];
    if (j >= 0) {
      const float2 yj = y[j];
      const float2 t = nn_term<L1>(yi, yj);
      fx += t.x; fy += t.y;
      if (ST) es += nn_stress<L1>(yi, yj);
    }
  }
  for (int q = 0; q < A.rn; ++q) {
    const int32_t k = A.rn_idx[i * A.rn + q];
    if (k >= 0) {
      const float2 yk = y[k];
      const float2 t = rn_term<L1>(yi, yk, A.c, A.eps);
      fx += t.x; fy += t.y;
      if (ST) es += rn_stress<L1>(yi, yk, (double)A.c);
      if (ARN) add_reaction(A, k, t);
    }
  }
  gather_segment<false, L1>(y, A.nn_src, ns, ne, yi, A.c, A.eps, fx, fy);
  if (!ARN && A.rn > 0)
    gather_segment<true, L1>(y, A.rn_src, A.rn_ptr[i], A.rn_ptr[i + 1], yi, A.c, A.eps, fx, fy);
  return make_float2(fx, fy);
}

// force on a vertex computed by a group of G aligned lanes (a whole
// wavefront for a hub, G = 64; four lanes for a light vertex of a small
// graph): the vertex's edge list (out-nn | out-rn | in-nn | in-rn) is split
// over the group's lanes round-robin, then reduced with a fixed butterfly
// over the group; every lane of the group returns the total.  r is the
// lane's rank in the group, [ns, ne) the vertex's nn in-edge segment.  With
// ST each lane adds the stress terms of its out-edges to its own es.
template <bool L1, bool ARN, bool ST, int G>
__device__ __forceinline__ float2 spread_force(const StepArgs &A, int64_t i, float2 yi, int r, int32_t ns,
                                               int32_t ne, double &es) {
  static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "a group is a power of two within a wavefront");
  const float2 *__restrict__ y = A.h;
  const int32_t rs = !ARN && A.rn > 0 ? A.rn_ptr[i] : 0, re = !ARN && A.rn > 0 ? A.rn_ptr[i + 1] : 0;
  const int32_t n_out = A.nn + A.rn, n_in_nn = ne - ns;
  const int32_t total = n_out + n_in_nn + (re - rs);
  float fx = 0.f, fy = 0.f;
  // four of a lane's edges at a time: their index and position loads are
  // issued together, the terms are still added in ascending edge order
  for (int32_t e0 = r; e0 < total; e0 += 4 * G) {
    int32_t other[4];
    int kind[4];   // 0 none, 1 nn, 2 rn
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t e = e0 + u * G;
      int32_t o = -1;
      int k = 0;
      if (e < total) {
        if (e < A.nn) {
          o = A.nn_idx[i * A.nn + e];
          k = 1;
        } else if (e < n_out) {
          o = A.rn_idx[i * A.rn + (e - A.nn)];
          k = 2;
        } else if (e < n_out + n_in_nn) {
          o = A.nn_src[ns + (e - n_out)];
          k = 1;
        } else {
          o = A.rn_src[rs + (e - n_out - n_in_nn)];
          k = 2;
        }
      }
      other[u] = o;
      kind[u] = o >= 0 ? k : 0;
    }
    float2 yo[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) yo[u] = kind[u] ? y[other[u]] : yi;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!kind[u]) continue;
      const float2 t = kind[u] == 1 ? nn_term<L1>(yi, yo[u]) : rn_term<L1>(yi, yo[u], A.c, A.eps);
      fx += t.x; fy += t.y;
      if (ST && e0 + u * G < n_out)
        es += kind[u] == 1 ? nn_stress<L1>(yi, yo[u]) : rn_stress<L1>(yi, yo[u], (double)A.c);
      // an rn out-edge (the only rn edges listed with ARN): its reaction by atomics
      if (ARN && kind[u] == 2) add_reaction(A, other[u], t);
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
  }
  return make_float2(fx, fy);
}

// v' = a v + b f, y' = y + v' (Adam: its moment update instead).  hi is the
// position the force was taken at (y itself unless OPT_NEST).  Returns the
// vertex's |v'|^2 - |v|^2 in FP64 for OPT_ADAPT (+inf when the tentative
// position is not finite, which forces a rejection); the non-finite flag is
// raised only for steps that are final.
template <int OPT>
__device__ __forceinline__ double apply_update(const StepArgs &A, int64_t i, float2 hi, float2 f) {
  constexpr bool NEST = OPT == OPT_NEST, ADAPT = OPT == OPT_ADAPT, ADAM = OPT == OPT_ADAM;
  const float2 yi = NEST ? A.y[i] : hi;
  const float2 v0 = A.v[i];
  float2 yn;
  float2 v;
  if (ADAM) {
    const float gx = -2.f * f.x, gy = -2.f * f.y;
    const float2 s0 = A.s2[i];
    const float c1 = A.adam->c1, c2 = A.adam->c2;
    v = make_float2(fmaf(A.beta1, v0.x, (1.f - A.beta1) * gx), fmaf(A.beta1, v0.y, (1.f - A.beta1) * gy));
    const float2 s1 = make_float2(fmaf(A.beta2, s0.x, (1.f - A.beta2) * gx * gx),
                                  fmaf(A.beta2, s0.y, (1.f - A.beta2) * gy * gy));
    yn = make_float2(yi.x - A.lr * (v.x / c1) / (A.eps_adam + sqrtf(s1.x / c2)),
                     yi.y - A.lr * (v.y / c1) / (A.eps_adam + sqrtf(s1.y / c2)));
    A.s2[i] = s1;
  } else {
    const float b = ADAPT ? *A.b_dev : A.b;
    // explicit fused multiply-adds: every variant rounds the update identically
    v = make_float2(fmaf(b, f.x, A.a * v0.x), fmaf(b, f.y, A.a * v0.y));
    yn = make_float2(yi.x + v.x, yi.y + v.y);
  }
  A.y_out[i] = yn;
  if (ADAPT) {
    A.v_out[i] = v;
  } else {
    A.v[i] = v;
  }
  if (NEST) A.h_out[i] = make_float2(fmaf(A.a, v.x, yn.x), fmaf(A.a, v.y, yn.y));
  const bool finite = isfinite(yn.x) && isfinite(yn.y);
  if (ADAPT) {
    if (!finite) return (double)INFINITY;
    return ((double)v.x * v.x + (double)v.y * v.y) - ((double)v0.x * v0.x + (double)v0.y * v0.y);
  }
  if (!finite) A.flags[FLAG_NONFINITE] = 1;
  return 0.0;
}

// fixed-order block sum of one double per thread (kDetBlock threads)
__device__ __forceinline__ void block_sum_store(double x, double *out) {
  __shared__ double lds[kDetBlock];
  lds[threadIdx.x] = x;
  __syncthreads();
  for (int s = kDetBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

// GRAD = true: out = s grad E = -2 s f with s = *gscale (1 when NULL), at
// A.h = A.y, stored through A.out_perm when set; with ST also each block's
// FP64 stress of its vertices' out-edges to A.e_part.  Otherwise one
// iteration (force + update).  No thread leaves before the block sums.
// ARN = true is pass 1 of the atomic mode: each vertex's own share (its nn
// edges both ways and its rn out-edges) goes to A.fown, the rn reactions to
// A.facc (A.fbuf outside the fixed range) by atomics; no update.
// G = lanes per light vertex (A.lanes): 1, or kSmallGraphLanes on graphs of
// fewer than kSmallGraphVertices vertices, where one lane per vertex leaves
// too few wavefronts to hide each lane's chain of dependent loads.
template <bool GRAD, bool L1, int OPT, bool ARN = false, bool ST = false, int G = 1>
__global__ void __launch_bounds__(kDetBlock) det_kernel(StepArgs A, float2 *out) {
  static_assert(!ST || GRAD, "the stress is accumulated by the gradient kernels only");
  static_assert(G == 1 || G == kSmallGraphLanes, "lanes per light vertex");
  double ke = 0.0, es = 0.0;
  if ((int32_t)blockIdx.x < A.heavy_blocks) {
    const int lane = threadIdx.x & 63;
    const int32_t h = (int32_t)blockIdx.x * kHeavyPerBlock + (int32_t)(threadIdx.x >> 6);
    if (h < A.n_heavy) {   // uniform over the wavefront
      const int64_t i = A.heavy[h];
      const float2 hi = A.h[i];
      const float2 f = spread_force<L1, ARN, ST, 64>(A, i, hi, lane, A.nn_ptr[i], A.nn_ptr[i + 1], es);
      if (lane == 0) {
        if (ARN) {
          A.fown[i] = f;
        } else if (GRAD) {
          const float g = -2.f * (A.gscale ? *A.gscale : 1.f);
          out[A.out_perm ? A.out_perm[i] : i] = make_float2(g * f.x, g * f.y);
        } else {
          ke = apply_update<OPT>(A, i, hi, f);
        }
      }
    }
  } else {
    // XCD-aware tiles: blocks are dealt to the XCDs round-robin, so block b
    // runs on XCD b % kXcds; each XCD is given one contiguous range of tiles,
    // keeping the positions its vertices gather from in its own L2
    // (a tile is kDetBlock / G consecutive vertices; with G > 1 the group
    // condition below is uniform over each group of G lanes)
    const int32_t lb = (int32_t)blockIdx.x - A.heavy_blocks;
    const int32_t tile = (lb % kXcds) * A.tiles_per_xcd + lb / kXcds;
    const int64_t i = (int64_t)tile * (kDetBlock / G) + threadIdx.x / G;
    const int r = (int)(threadIdx.x % G);
    if (tile < A.light_tiles && i < A.M) {
      const int32_t ns = A.nn_ptr[i], ne = A.nn_ptr[i + 1];
      if (ne - ns <= A.heavy_deg) {   // else served by a heavy wavefront
        const float2 hi = A.h[i];
        float2 f;
        if constexpr (G == 1) f = light_force<L1, ARN, ST>(A, i, hi, ns, ne, es);
        else f = spread_force<L1, ARN, ST, G>(A, i, hi, r, ns, ne, es);
        if (r != 0) {
          // the group's leader stores the result
        } else if (ARN) {
          A.fown[i] = f;
        } else if (GRAD) {
          const float g = -2.f * (A.gscale ? *A.gscale : 1.f);
          out[A.out_perm ? A.out_perm[i] : i] = make_float2(g * f.x, g * f.y);
        } else {
          ke = apply_update<OPT>(A, i, hi, f);
        }
      }
    }
  }
  if (OPT == OPT_ADAPT) block_sum_store(ke, A.ke_part + blockIdx.x);
  if (ST) block_sum_store(es, A.e_part + blockIdx.x);
}

__global__ void heavy_list_kernel(const int32_t *__restrict__ nn_ptr, int64_t M, int heavy_deg, int32_t *list,
                                  int32_t *count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  if (nn_ptr[i + 1] - nn_ptr[i] > heavy_deg) list[atomicAdd(count, 1)] = (int32_t)i;
}

// the force on vertex i after pass 1 of the atomic mode: own share, then
// the fixed-point reactions, then the float ones; the accumulators cleared.
// The float accumulator is read (and cleared) only when the flag of this
// iteration's slot is set; the other slot is cleared here for the next
// iteration.  A flag left set from an earlier iteration only costs a read
// of zeros, while every pass 1 that used fbuf has set the slot its pass 2
// reads: nothing between them clears that slot.
__device__ __forceinline__ float2 gather_reactions(const StepArgs &A, int64_t i) {
  const float2 fo = A.fown[i];
  if (A.rn == 0) return fo;
  if (i == 0) A.fflag[A.fpar ^ 1] = 0;
  const float2 fx = fixed_reactions(A.facc[i], A.rx_unit);
  A.facc[i] = 0;
  float2 f = make_float2(fo.x + fx.x, fo.y + fx.y);
  if (A.fflag[A.fpar]) {
    const float2 fr = A.fbuf[i];
    A.fbuf[i] = make_float2(0.f, 0.f);
    f = make_float2(f.x + fr.x, f.y + fr.y);
  }
  return f;
}

// update after the scatter pass; in place (y_out == y), H rewritten in place
template <int OPT>
__global__ void __launch_bounds__(kBlock) atomic_update_kernel(StepArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 f = gather_reactions(A, i);
  (void)apply_update<OPT>(A, i, OPT == OPT_NEST ? make_float2(0.f, 0.f) : A.y[i], f);
}

__global__ void __launch_bounds__(kBlock) atomic_grad_out_kernel(StepArgs A, float2 *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 f = gather_reactions(A, i);
  const float g = -2.f * (A.gscale ? *A.gscale : 1.f);
  out[A.out_perm ? A.out_perm[i] : i] = make_float2(g * f.x, g * f.y);
}

// rr->part[b]: the largest count of block b's stride of cnt[0..M)
__global__ void __launch_bounds__(kBlock) range_parts_kernel(const int32_t *__restrict__ cnt, int64_t M,
                                                             ReactionRange *rr) {
  __shared__ int32_t lds[kBlock];
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < M; i += (int64_t)gridDim.x * kBlock)
    m = max(m, cnt[i]);
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] = max(lds[threadIdx.x], lds[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) rr->part[blockIdx.x] = lds[0];
}

// rr->cap = 2^(30 - ceil(log2 K)), K the largest of the nparts partial maxima
// (at least 1): K reactions of at most cap units each sum to at most 2^30
__global__ void __launch_bounds__(kRangeParts) range_cap_kernel(ReactionRange *rr, int nparts) {
  __shared__ int32_t lds[kRangeParts];
  lds[threadIdx.x] = (int)threadIdx.x < nparts ? rr->part[threadIdx.x] : 0;
  __syncthreads();
  for (int s = kRangeParts / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] = max(lds[threadIdx.x], lds[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t k = (uint32_t)max(lds[0], 1);
    const int ceil_log2 = 32 - __clz((int)(k - 1u));
    rr->cap = ldexpf(1.f, 30 - ceil_log2);
  }
}

__global__ void adam_prep_kernel(AdamState *st, float beta1, float beta2) {
  const int64_t t = st->t + 1;
  st->t = t;
  st->c1 = 1.f - powf(beta1, (float)t);
  st->c2 = 1.f - powf(beta2, (float)t);
}

// H = Y + a V (the look-ahead positions of the Nesterov variant)
__global__ void lookahead_kernel(const float2 *__restrict__ y, const float2 *__restrict__ v, float a, int64_t M,
                                 float2 *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float2 yi = y[i], vi = v[i];
  h[i] = make_float2(yi.x + a * vi.x, yi.y + a * vi.y);
}

// accept / reject of a tentative step: dT = the fixed-order sum of the block
// partials; kept when finite and |dT| <= tau, else b *= (dT < -tau ? g1 : g2)
constexpr int kDecideThreads = 1024;

__global__ void __launch_bounds__(kDecideThreads) adapt_decide_kernel(const double *__restrict__ part, int nparts,
                                                                      double tau, float g1, float g2,
                                                                      AdaptState *st) {
  __shared__ double lds[kDecideThreads];
  double x = 0.0;
  // the loads of eight terms fly together; they are still added in order
#pragma unroll 8
  for (int p = threadIdx.x; p < nparts; p += kDecideThreads) x += part[p];
  lds[threadIdx.x] = x;
  __syncthreads();
  for (int s = kDecideThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dT = lds[0];
    const bool keep = isfinite(dT) && fabs(dT) <= tau;
    st->dT = dT;
    st->reject = keep ? 0 : 1;
    if (keep) {
      st->kept += 1;
    } else {
      st->b = st->b * (dT < -tau ? g1 : g2);
      st->rejected += 1;
    }
  }
}

// after a rejection the next state is the current one again (a small
// grid-stride launch: it costs next to nothing when the step was kept)
__global__ void adapt_commit_kernel(const AdaptState *__restrict__ st, const float2 *__restrict__ y,
                                    const float2 *__restrict__ v, int64_t M, float2 *__restrict__ y_next,
                                    float2 *__restrict__ v_next) {
  if (!st->reject) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    y_next[i] = y[i];
    v_next[i] = v[i];
  }
}

}  // namespace

hipError_t launch_lookahead(const float2 *y, const float2 *v, float a, int64_t M, float2 *h, hipStream_t s) {
  lookahead_kernel<<<grid_for(M), kBlock, 0, s>>>(y, v, a, M, h);
  return hipGetLastError();
}

hipError_t launch_adam_prep(AdamState *st, float beta1, float beta2, hipStream_t s) {
  adam_prep_kernel<<<1, 1, 0, s>>>(st, beta1, beta2);
  return hipGetLastError();
}

hipError_t launch_adapt_decide(const double *part, int nparts, double tau, float g1, float g2, AdaptState *st,
                               hipStream_t s) {
  adapt_decide_kernel<<<1, kDecideThreads, 0, s>>>(part, nparts, tau, g1, g2, st);
  return hipGetLastError();
}

hipError_t launch_adapt_commit(const AdaptState *st, const float2 *y, const float2 *v, int64_t M, float2 *y_next,
                               float2 *v_next, hipStream_t s) {
  const unsigned g = grid_for(M) < 1024u ? grid_for(M) : 1024u;
  adapt_commit_kernel<<<g, kBlock, 0, s>>>(st, y, v, M, y_next, v_next);
  return hipGetLastError();
}

unsigned det_grid(const StepArgs &a) { return (unsigned)(a.heavy_blocks + kXcds * a.tiles_per_xcd); }

hipError_t launch_heavy_list(const int32_t *nn_ptr, int64_t M, int heavy_deg, int32_t *list, int32_t *count,
                             hipStream_t s) {
  heavy_list_kernel<<<grid_for(M), kBlock, 0, s>>>(nn_ptr, M, heavy_deg, list, count);
  return hipGetLastError();
}

// one deterministic launch, with the lanes per light vertex of the shape
template <bool GRAD, bool L1, int OPT, bool ARN = false, bool ST = false>
void launch_det(const StepArgs &a, float2 *out, hipStream_t s) {
  if (a.lanes == kSmallGraphLanes)
    det_kernel<GRAD, L1, OPT, ARN, ST, kSmallGraphLanes><<<det_grid(a), kDetBlock, 0, s>>>(a, out);
  else
    det_kernel<GRAD, L1, OPT, ARN, ST, 1><<<det_grid(a), kDetBlock, 0, s>>>(a, out);
}

template <bool L1>
void launch_det_opt(const StepArgs &a, hipStream_t s) {
  switch (a.opt) {
    case OPT_NEST: launch_det<false, L1, OPT_NEST>(a, nullptr, s); break;
    case OPT_ADAPT: launch_det<false, L1, OPT_ADAPT>(a, nullptr, s); break;
    case OPT_ADAM: launch_det<false, L1, OPT_ADAM>(a, nullptr, s); break;
    default: launch_det<false, L1, OPT_PLAIN>(a, nullptr, s); break;
  }
}

hipError_t launch_step_det(const StepArgs &a, hipStream_t s) {
  if (a.l1) launch_det_opt<true>(a, s);
  else launch_det_opt<false>(a, s);
  return hipGetLastError();
}

hipError_t launch_step_atomic(const StepArgs &a, hipStream_t s) {
  if (a.l1) launch_det<false, true, OPT_PLAIN, true>(a, nullptr, s);
  else launch_det<false, false, OPT_PLAIN, true>(a, nullptr, s);
  if (a.opt == OPT_NEST) atomic_update_kernel<OPT_NEST><<<grid_for(a.M), kBlock, 0, s>>>(a);
  else atomic_update_kernel<OPT_PLAIN><<<grid_for(a.M), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_grad_det(const StepArgs &a, float2 *out, hipStream_t s) {
  if (a.e_part) {
    if (a.l1) launch_det<true, true, OPT_PLAIN, false, true>(a, out, s);
    else launch_det<true, false, OPT_PLAIN, false, true>(a, out, s);
  } else {
    if (a.l1) launch_det<true, true, OPT_PLAIN>(a, out, s);
    else launch_det<true, false, OPT_PLAIN>(a, out, s);
  }
  return hipGetLastError();
}

hipError_t launch_grad_atomic(const StepArgs &a, float2 *out, hipStream_t s) {
  if (a.l1) launch_det<false, true, OPT_PLAIN, true>(a, nullptr, s);
  else launch_det<false, false, OPT_PLAIN, true>(a, nullptr, s);
  atomic_grad_out_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a, out);
  return hipGetLastError();
}

hipError_t launch_reaction_range(const int32_t *cnt, int64_t M, ReactionRange *rr, hipStream_t s) {
  const unsigned g = grid_for(M);
  const int nparts = g < (unsigned)kRangeParts ? (int)g : kRangeParts;
  range_parts_kernel<<<nparts, kBlock, 0, s>>>(cnt, M, rr);
  range_cap_kernel<<<1, kRangeParts, 0, s>>>(rr, nparts);
  return hipGetLastError();
}

}  // namespace ivhd
