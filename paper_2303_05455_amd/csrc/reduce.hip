// FP64 stress of Eq. ivhd_cost_function for reporting:
//   E = sum_i [ sum_{j in O_nn(i)} d_ij^2 + c * sum_{k in O_rn(i)} (1 - d_ik)^2 ]
// with d the Euclidean distance, or |dx| + |dy| for the l1 variant.
// Each thread sums the out-edges of one vertex in double precision (from the
// FP32 positions, widened before subtracting), each block reduces its 256
// values in a fixed tree, and a single block adds the block sums in a fixed
// order -- so the result is bitwise reproducible.
#include "ivhd_internal.h"

namespace ivhd {
namespace {

constexpr int kStressBlock = 256;

template <bool L1>
__global__ void __launch_bounds__(kStressBlock)
stress_partial_kernel(const float2 *__restrict__ y, int64_t M, const int32_t *__restrict__ nn_idx,
                      int nn, const int32_t *__restrict__ rn_idx, int rn, double c,
                      double *__restrict__ partials) {
  __shared__ double lds[kStressBlock];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < M) {
    const float2 yi = y[i];
    for (int q = 0; q < nn; ++q) {
      const int32_t j = nn_idx[i * nn + q];
      if (j < 0) continue;
      const float2 yj = y[j];
      const double dx = (double)yi.x - (double)yj.x, dy = (double)yi.y - (double)yj.y;
      if (L1) {
        const double d = fabs(dx) + fabs(dy);
        e += d * d;
      } else {
        e += dx * dx + dy * dy;
      }
    }
    for (int q = 0; q < rn; ++q) {
      const int32_t k = rn_idx[i * rn + q];
      if (k < 0) continue;
      const float2 yk = y[k];
      const double dx = (double)yi.x - (double)yk.x, dy = (double)yi.y - (double)yk.y;
      const double d = L1 ? fabs(dx) + fabs(dy) : sqrt(dx * dx + dy * dy);
      e += c * (1.0 - d) * (1.0 - d);
    }
  }
  lds[threadIdx.x] = e;
  __syncthreads();
  for (int s = kStressBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = lds[0];
}

// one block: thread t adds partials t, t + kFinalBlock, t + 2 kFinalBlock, ...
// in that order (eight loads in flight), then a fixed tree over the threads
constexpr int kFinalBlock = 1024;

__global__ void __launch_bounds__(kFinalBlock)
stress_final_kernel(const double *__restrict__ partials, int nparts, double *out) {
  __shared__ double lds[kFinalBlock];
  double e = 0.0;
  for (int base = threadIdx.x; base < nparts; base += 8 * kFinalBlock) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = base + u * kFinalBlock;
      v[u] = p < nparts ? partials[p] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) e += v[u];
  }
  lds[threadIdx.x] = e;
  __syncthreads();
  for (int s = kFinalBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

// out may equal x
__global__ void scale_f32_kernel(const float *x, int64_t n, const float *scale, float *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = *scale * x[k];
}

}  // namespace

hipError_t launch_stress_final(const double *partials, int nparts, double *out, hipStream_t s) {
  stress_final_kernel<<<1, kFinalBlock, 0, s>>>(partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_scale_f32(const float *x, int64_t n, const float *scale, float *out, hipStream_t s) {
  if (n > 0) scale_f32_kernel<<<grid_for(n, kStressBlock), kStressBlock, 0, s>>>(x, n, scale, out);
  return hipGetLastError();
}

int stress_partials(int64_t M) { return (int)grid_for(M, kStressBlock); }

hipError_t launch_stress(const float2 *y, int64_t M, const int32_t *nn_idx, int nn,
                         const int32_t *rn_idx, int rn, double c, int metric, double *partials, int nparts,
                         double *out, hipStream_t s) {
  if (metric == 1)
    stress_partial_kernel<true><<<(unsigned)nparts, kStressBlock, 0, s>>>(y, M, nn_idx, nn, rn_idx, rn, c,
                                                                         partials);
  else
    stress_partial_kernel<false><<<(unsigned)nparts, kStressBlock, 0, s>>>(y, M, nn_idx, nn, rn_idx, rn, c,
                                                                          partials);
  stress_final_kernel<<<1, kFinalBlock, 0, s>>>(partials, nparts, out);
  return hipGetLastError();
}

}  // namespace ivhd
