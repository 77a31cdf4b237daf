// k_util.hip -- image initialisation and the Philox parity hook.
#include "cfs_device.hpp"
#include "cfs_host.hpp"

namespace cfs {

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  // scalar head up to 16-byte alignment, 16-byte stores over the body,
  // scalar tail
  size_t head = (16 - (reinterpret_cast<uintptr_t>(p) & 15)) / 4 % 4;
  if (head > n) head = n;
  if (i < head) p[i] = v;
  const size_t n4 = (n - head) / 4;
  uint4 *p4 = reinterpret_cast<uint4 *>(p + head);
  for (size_t j = i; j < n4; j += stride) p4[j] = make_uint4(v, v, v, v);
  for (size_t j = head + n4 * 4 + i; j < n; j += stride) p[j] = v;
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, size_t n, unsigned long long v) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t j = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride)
    p[j] = v;
}

static unsigned fill_blocks(size_t n) {
  const size_t want = (n + 1023) / 1024;
  return static_cast<unsigned>(want < 1 ? 1 : (want > 8192 ? 8192 : want));
}

hipError_t launch_clear_u32(uint32_t *p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n / 4 + 1)), dim3(256), 0, s, p, n, 0u);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_philox_dump(uint32_t k0, uint32_t k1, const uint32_t *__restrict__ ctrs,
                              uint32_t *__restrict__ out, uint64_t n) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = reinterpret_cast<const uint4 *>(ctrs)[i];
  const Block4 b = philox10(c.x, c.y, c.z, c.w, k0, k1);
  reinterpret_cast<uint4 *>(out)[i] = make_uint4(b.w0, b.w1, b.w2, b.w3);
}

hipError_t launch_philox_dump(uint32_t k0, uint32_t k1, const uint32_t *ctrs, uint32_t *out,
                              uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_philox_dump, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, k0, k1,
                     ctrs, out, n);
  return hipGetLastError();
}

}  // namespace cfs
