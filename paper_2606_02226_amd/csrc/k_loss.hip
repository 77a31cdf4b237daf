// k_loss.hip -- the L2 image loss of the fitting loop and its gradient
// (Section 4: fitting a primitive's distribution with autodiff-like tools).
//
// L = sum_i (D_i - D*_i)^2 in FP64 and dL/dD_i = 2 (D_i - D*_i) rounded once
// to FP32.  The
// grid depends only on n, every thread sums a fixed strided set of elements,
// and both reductions run in a fixed order, so L is bit-reproducible.
#include "cfs_host.hpp"

namespace cfs {

constexpr int kLossBlock = 256;
constexpr uint32_t kLossMaxBlocks = 1024;

uint32_t loss_blocks(uint64_t n) {
  const uint64_t want = (n + kLossBlock * 8 - 1) / (kLossBlock * 8);
  return static_cast<uint32_t>(want < 1 ? 1 : (want > kLossMaxBlocks ? kLossMaxBlocks : want));
}

// Fixed-order sum of one value per thread of a kLossBlock workgroup; the
// result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds) {
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int s = kLossBlock / 2; s > 0; s >>= 1) {
    if (tid < s) lds[tid] += lds[tid + s];
    __syncthreads();
  }
  return lds[0];
}

__global__ __launch_bounds__(kLossBlock) void k_l2_partial(const float *__restrict__ d,
                                                           const float *__restrict__ target,
                                                           uint64_t n, float *__restrict__ grad,
                                                           double *__restrict__ partial) {
  __shared__ double lds[kLossBlock];
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kLossBlock;
  double acc = 0.0;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kLossBlock + threadIdx.x; i < n;
       i += stride) {
    // the difference of two floats is exact in double
    const double diff = static_cast<double>(d[i]) - static_cast<double>(target[i]);
    if (grad) grad[i] = static_cast<float>(2.0 * diff);
    acc += diff * diff;
  }
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kLossBlock) void k_l2_final(const double *__restrict__ partial,
                                                         uint32_t blocks, double *__restrict__ loss) {
  __shared__ double lds[kLossBlock];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < blocks; i += kLossBlock) acc += partial[i];
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) loss[0] = s;
}

hipError_t launch_l2_loss(const float *d, const float *target, uint64_t n, float *grad,
                          double *loss, double *partial, hipStream_t s) {
  const uint32_t blocks = loss_blocks(n);
  hipLaunchKernelGGL(k_l2_partial, dim3(blocks), dim3(kLossBlock), 0, s, d, target, n, grad,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(kLossBlock), 0, s, partial, blocks, loss);
  return hipGetLastError();
}

}  // namespace cfs
