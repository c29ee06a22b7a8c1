// One IVHD iteration on gfx950 (Sec. "Force directed", Eq.
// force_directed_update, with the force of Eq. eq13 taken as -1/2 grad of
// Eq. ivhd_cost_function):
//
//   every edge incident to vertex i, whichever way it points, acts on i with
//     nn edge:  -(y_i - y_o)
//     rn edge:  c (1 - d) (y_i - y_o) / max(d, eps),   d = |y_i - y_o|
//   f_i = sum of those;   v_i <- a v_i + b f_i ;   y_i <- y_i + v_i
//
// Deterministic mode: one thread per vertex gathers its out-edges (rows of
// nn_idx / rn_idx) and its in-edges (the transposed lists, sources
// ascending) in a fixed order -- out-nn, out-rn, in-nn, in-rn -- then
// updates v in place and writes y to the other half of a ping-pong pair, so
// no thread reads a position another thread has already moved.  Force and
// update are fused: one kernel per iteration, no force array in memory.
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

__device__ __forceinline__ float2 gather_force(const StepArgs &A, int64_t i, float2 yi) {
  const float2 *__restrict__ y = A.y;
  float fx = 0.f, fy = 0.f;
  for (int q = 0; q < A.nn; ++q) {
    const int32_t j = A.nn_idx[i * A.nn + q];
    if (j >= 0) {
      float2 t = nn_term(yi, y[j]);
      fx += t.x; fy += t.y;
    }
  }
  for (int q = 0; q < A.rn; ++q) {
    const int32_t k = A.rn_idx[i * A.rn + q];
    float2 t = rn_term(yi, y[k], A.c, A.eps);
    fx += t.x; fy += t.y;
  }
  for (int32_t p = A.nn_ptr[i], e = A.nn_ptr[i + 1]; p < e; ++p) {
    float2 t = nn_term(yi, y[A.nn_src[p]]);
    fx += t.x; fy += t.y;
  }
  if (A.rn > 0) {
    for (int32_t p = A.rn_ptr[i], e = A.rn_ptr[i + 1]; p < e; ++p) {
      float2 t = rn_term(yi, y[A.rn_src[p]], A.c, A.eps);
      fx += t.x; fy += t.y;
    }
  }
  return make_float2(fx, fy);
}

__global__ void __launch_bounds__(kBlock) step_det_kernel(StepArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 yi = A.y[i];
  const float2 f = gather_force(A, i, yi);
  const float2 v0 = A.v[i];
  const float2 v = make_float2(A.a * v0.x + A.b * f.x, A.a * v0.y + A.b * f.y);
  const float2 yn = make_float2(yi.x + v.x, yi.y + v.y);
  A.v[i] = v;
  A.y_out[i] = yn;
  if (!(isfinite(yn.x) && isfinite(yn.y))) A.flags[FLAG_NONFINITE] = 1;
}

__global__ void __launch_bounds__(kBlock) grad_det_kernel(StepArgs A, float2 *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.M) return;
  const float2 f = gather_force(A, i, A.y[i]);
  out[i] = make_float2(-2.f * f.x, -2.f * f.y);
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
  const float2 v0 = A.v[i];
  const float2 v = make_float2(A.a * v0.x + A.b * f.x, A.a * v0.y + A.b * f.y);
  const float2 yi = A.y[i];
  const float2 yn = make_float2(yi.x + v.x, yi.y + v.y);
  A.v[i] = v;
  A.y_out[i] = yn;
  if (!(isfinite(yn.x) && isfinite(yn.y))) A.flags[FLAG_NONFINITE] = 1;
}

__global__ void __launch_bounds__(kBlock) atomic_grad_out_kernel(float2 *fbuf, int64_t M, float2 *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float2 f = fbuf[i];
  fbuf[i] = make_float2(0.f, 0.f);
  out[i] = make_float2(-2.f * f.x, -2.f * f.y);
}

}  // namespace

hipError_t launch_step_det(const StepArgs &a, hipStream_t s) {
  step_det_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_step_atomic(const StepArgs &a, hipStream_t s) {
  scatter_force_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  atomic_update_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_grad_det(const StepArgs &a, float2 *out, hipStream_t s) {
  grad_det_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a, out);
  return hipGetLastError();
}

hipError_t launch_grad_atomic(const StepArgs &a, float2 *out, hipStream_t s) {
  scatter_force_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a);
  atomic_grad_out_kernel<<<grid_for(a.M), kBlock, 0, s>>>(a.fbuf, a.M, out);
  return hipGetLastError();
}

}  // namespace ivhd
