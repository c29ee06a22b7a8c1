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
//     kHeavyDegree a whole wavefront: the 64 lanes stride over its edge list
//     and a fixed xor-butterfly adds their partial sums;
//   * the other blocks give each remaining vertex one thread, which issues
//     its in-edge gathers four at a time so several loads are in flight.
// Both orders of summation are fixed, so results are bitwise reproducible.
//
// Atomic mode: pass 1, one thread per vertex, walks its out-edges, keeps its
// own share in registers and adds each reaction to the other end with a
// float atomic; pass 2 applies the update and clears the accumulator.
#include "ivhd_internal.h"

namespace ivhd {
namespace {

__device__ __forceinline__ float2 nn_term(float2 yi, float2 yo) {
  return make_float2(yo.x - yi.x, yo.y - yi.y);
}

__device__ __forceinline__ float2 rn_term(float2 yi, float2 yo, float c, float eps) {
  const float dx = yi.x - yo.x, dy = yi.y - yo.y;
  const float d = sqrtf(dx * dx + dy * dy);
  const float s = c * (1.0f - d) / fmaxf(d, eps);
  return make_float2(s * dx, s * dy);
}

// in-edge segment [s, e) of a light vertex, four gathers in flight at a time;
// the terms are still added one by one in ascending order
template <bool RN>
__device__ __forceinline__ void gather_segment(const float2 *__restrict__ y, const int32_t *__restrict__ src,
                                               int32_t s, int32_t e, float2 yi, float c, float eps,
                                               float &fx, float &fy) {
  int32_t p = s;
  for (; p + 4 <= e; p += 4) {
    const int32_t j0 = src[p], j1 = src[p + 1], j2 = src[p + 2], j3 = src[p + 3];
    const float2 y0 = y[j0], y1 = y[j1], y2 = y[j2], y3 = y[j3];
    float2 t;
    t = RN ? rn_term(yi, y0, c, eps) : nn_term(yi, y0); fx += t.x; fy += t.y;
    t = RN ? rn_term(yi, y1, c, eps) : nn_term(yi, y1); fx += t.x; fy += t.y;
    t = RN ? rn_term(yi, y2, c, eps) : nn_term(yi, y2); fx += t.x; fy += t.y;
    t = RN ? rn_term(yi, y3, c, eps) : nn_term(yi, y3); fx += t.x; fy += t.y;
  }
  for (; p < e; ++p) {
    const float2 t = RN ? rn_term(yi, y[src[p]], c, eps) : nn_term(yi, y[src[p]]);
    fx += t.x; fy += t.y;
  }
}

// force on a light vertex: out-nn, out-rn, in-nn, in-rn, in that order
__device__ __forceinline__ float2 light_force(const StepArgs &A, int64_t i, float2 yi, int32_t ns,
                                              int32_t ne) {
  const float2 *__restrict__ y = A.y;
  float fx = 0.f, fy = 0.f;
  for (int q = 0; q < A.nn; ++q) {
    const int32_t j = A.nn_idx[i * A.nn + q];
    if (j >= 0) {
      const float2 t = nn_term(yi, y[j]);
      fx += t.x; fy += t.y;
    }
  }
  for (int q = 0; q < A.rn; ++q) {
    const int32_t k = A.rn_idx[i * A.rn + q];
    if (k >= 0) {
      const float2 t = rn_term(yi, y[k], A.c, A.eps);
      fx += t.x; fy += t.y;
    }
  }
  gather_segment<false>(y, A.nn_src, ns, ne, yi, A.c, A.eps, fx, fy);
  if (A.rn > 0) gather_segment<true>(y, A.rn_src, A.rn_ptr[i], A.rn_ptr[i + 1], yi, A.c, A.eps, fx, fy);
  return make_float2(fx, fy);
}

// force on a heavy vertex, computed by a whole wavefront: the vertex's edge
// list (out-nn | out-rn | in-nn | in-rn) is split over the lanes round-robin,
// then reduced with a fixed butterfly; every lane returns the total
__device__ __forceinline__ float2 heavy_force(const StepArgs &A, int64_t i, float2 yi, int lane) {
  const float2 *__restrict__ y = A.y;
  const int32_t ns = A.nn_ptr[i], ne = A.nn_ptr[i + 1];
  const int32_t rs = A.rn > 0 ? A.rn_ptr[i] : 0, re = A.rn > 0 ? A.rn_ptr[i + 1] : 0;
  const int32_t n_out = A.nn + A.rn, n_in_nn = ne - ns;
  const int32_t total = n_out + n_in_nn + (re - rs);
  float fx = 0.f, fy = 0.f;
  for (int32_t e = lane; e < total; e += 64) {
    float2 t;
    if (e < A.nn) {
      const int32_t j = A.nn_idx[i * A.nn + e];
      t = j >= 0 ? nn_term(yi, y[j]) : make_float2(0.f, 0.f);
    } else if (e < n_out) {
      const int32_t k = A.rn_idx[i * A.rn + (e - A.nn)];
      t = k >= 0 ? rn_term(yi, y[k], A.c, A.eps) : make_float2(0.f, 0.f);
    } else if (e < n_out + n_in_nn) {
      t = nn_term(yi, y[A.nn_src[ns + (e - n_out)]]);
    } else {
      t = rn_term(yi, y[A.rn_src[rs + (e - n_out - n_in_nn)]], A.c, A.eps);
    }
    fx += t.x; fy += t.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
  }
  return make_float2(fx, fy);
}

__device__ __forceinline__ void apply_update(const StepArgs &A, int64_t i, float2 yi, float2 f) {
  const float2 v0 = A.v[i];
  const float2 v = make_float2(A.a * v0.x + A.b * f.x, A.a * v0.y + A.b * f.y);
  const float2 yn = make_float2(yi.x + v.x, yi.y + v.y);
  A.v[i] = v;
  A.y_out[i] = yn;
  if (!(isfinite(yn.x) && isfinite(yn.y))) A.flags[FLAG_NONFINITE] = 1;
}

// GRAD = false: one iteration (force + update); GRAD = true: out = s grad E = -2 s f
// with s = *gscale (1 when NULL)
template <bool GRAD>
__global__ void __launch_bounds__(kBlock) det_kernel(StepArgs A, float2 *out) {
  if ((int32_t)blockIdx.x < A.heavy_blocks) {
    const int lane = threadIdx.x & 63;
    const int32_t h = (int32_t)blockIdx.x * kHeavyPerBlock + (int32_t)(threadIdx.x >> 6);
    if (h >= A.n_heavy) return;
    const int64_t i = A.heavy[h];
    const float2 yi = A.y[i];
    const float2 f = heavy_force(A, i, yi, lane);
    if (lane == 0) {
      if (GRAD) {
        const float g = -2.f * (A.gscale ? *A.gscale : 1.f);
        out[i] = make_float2(g * f.x, g * f.y);
      } else {
        apply_update(A, i, yi, f);
      }
    }
    return;
  }
  // XCD-aware tiles: blocks are dealt to the XCDs round-robin, so block b runs
  // on XCD b % kXcds; each XCD is given one contiguous range of tiles, keeping
  // the positions its vertices gather from in its own L2
  const int32_t lb = (int32_t)blockIdx.x - A.heavy_blocks;
  const int32_t tile = (lb % kXcds) * A.tiles_per_xcd + lb / kXcds;
  if (tile >= A.light_tiles) return;
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  if (i >= A.M) return;
  const int32_t ns = A.nn_ptr[i], ne = A.nn_ptr[i + 1];
  if (ne - ns > kHeavyDegree) return;   // served by a heavy wavefront
  const float2 yi = A.y[i];
  const float2 f = light_force(A, i, yi, ns, ne);
  if (GRAD) {
    const float g = -2.f * (A.gscale ? *A.gscale : 1.f);
    out[i] = make_float2(g * f.x, g * f.y);
  } else {
    apply_update(A, i, yi, f);
  }
}

__global__ void heavy_list_kernel(const int32_t *__restrict__ nn_ptr, int64_t M, int32_t *list,
                                  int32_t *count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  if (nn_ptr[i + 1] - nn_ptr[i] > kHeavyDegree) list[atomicAdd(count, 1)] = (int32_t)i;
}

__global__ void __launch_bounds__(kBlock) scatter_force_kernel(StepArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 *__restrict__ y = A.y;
  const float2 yi = y[i];
  float fx = 0.f, fy = 0.f;
  for (int q = 0; q < A.nn; ++q) {
    const int32_t j = A.nn_idx[i * A.nn + q];
    if (j >= 0) {
      float2 t = nn_term(yi, y[j]);
      fx += t.x; fy += t.y;
      unsafeAtomicAdd(&A.fbuf[j].x, -t.x);
      unsafeAtomicAdd(&A.fbuf[j].y, -t.y);
    }
  }
  for (int q = 0; q < A.rn; ++q) {
    const int32_t k = A.rn_idx[i * A.rn + q];
    float2 t = rn_term(yi, y[k], A.c, A.eps);
    fx += t.x; fy += t.y;
    unsafeAtomicAdd(&A.fbuf[k].x, -t.x);
    unsafeAtomicAdd(&A.fbuf[k].y, -t.y);
  }
  unsafeAtomicAdd(&A.fbuf[i].x, fx);
  unsafeAtomicAdd(&A.fbuf[i].y, fy);
}

__global__ void __launch_bounds__(kBlock) atomic_update_kernel(StepArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 f = A.fbuf[i];
  A.fbuf[i] = make_float2(0.f, 0.f);
  apply_update(A, i, A.y[i], f);
}

__global__ void __launch_bounds__(kBlock) atomic_grad_out_kernel(float2 *fbuf, int64_t M, const float *gscale,
                                                                float2 *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float2 f = fbuf[i];
  fbuf[i] = make_float2(0.f, 0.f);
  const float g = -2.f * (gscale ? *gscale : 1.f);
  out[i] = make_float2(g * f.x, g * f.y);
}

unsigned det_grid(const StepArgs &a) { return (unsigned)(a.heavy_blocks + kXcds * a.tiles_per_xcd); }

}  // namespace

hipError_t launch_heavy_list(const int32_t *nn_ptr, int64_t M, int32_t *list, int32_t *count,
                             hipStream_t s) {
  heavy_list_kernel<<<grid_for(M), kBlock, 0, s>>>(nn_ptr, M, list, count);
  return hipGetLastError();
}

hipError_t launch_step_det(const StepArgs &a, hipStream_t s) {
  det_kernel<false><<<det_grid(a), kBlock, 0, s>>>(a, nullptr);
  return hipGetLastError();
}

hipError_t launch_step_atomic(const StepArgs &a, hipStream_t s) {
  scatter_force_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  atomic_update_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_grad_det(const StepArgs &a, float2 *out, hipStream_t s) {
  det_kernel<true><<<det_grid(a), kBlock, 0, s>>>(a, out);
  return hipGetLastError();
}

hipError_t launch_grad_atomic(const StepArgs &a, float2 *out, hipStream_t s) {
  scatter_force_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  atomic_grad_out_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a.fbuf, a.M, a.gscale, out);
  return hipGetLastError();
}

}  // namespace ivhd
