// k_microbench.hip -- ceiling probes for the rooflines of the chaos game.
//
// The splat is an atomic histogram (Section 1: every iterate colours its
// pixel; Section 4: density estimation needs atomic operations, which can
// limit performance), so the rates that bound it are not published figures
// but those of the atomics themselves.  These kernels measure, on the same
// chip and with the same operation types as the splats:
//   copy       device-to-device copy with 16-byte vectors (HBM read + write);
//   dev_add    uniformly random u32 atomic adds into a device working set;
//   dev_min    uniformly random u64 atomic minima into a device working set;
//   lds_add    uniformly random u32 atomic adds into 64 KiB of LDS per
//              workgroup (the count accumulate's tile);
//   lds_add64  uniformly random u64 atomic adds into 64 KiB of LDS (the
//              Gaussian accumulate's fixed-point tap sums);
//   lds_min    uniformly random u64 atomic minima into 64 KiB of LDS (the
//              depth accumulate's key tile);
//   philox     Philox4x32-10 blocks (the chaos game's random numbers);
//   runs       reads of runs of 128, 512 or 2048 bytes at uniformly random
//              16-byte-aligned places in a large buffer, a group of lanes
//              per run and 16 bytes per lane, four runs in flight per group
//              (the accumulates read each chunk's run of their tile so).
// Addresses come from a per-lane linear congruential sequence (one 32-bit
// multiply-add per operation) scaled to the working set by a high multiply,
// so the address arithmetic is small next to the operation it feeds.  The
// caller times a call with events on its stream.
#include "cfs.h"
#include "cfs_api_internal.hpp"
#include "cfs_device.hpp"
#include "cfs_host.hpp"

namespace cfs {

namespace {

constexpr int kMbBlock = 256;
constexpr uint32_t kMbGrid = 4096;  // 16 workgroups per compute unit of MI355X
constexpr uint32_t kLcgMul = 1664525u, kLcgAdd = 1013904223u;

__device__ __forceinline__ uint32_t lane_seed() {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  return g * 0x9E3779B9u + 0x7F4A7C15u;
}

__global__ __launch_bounds__(kMbBlock) void k_mb_copy(const uint4 *__restrict__ src,
                                                      uint4 *__restrict__ dst, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

__global__ __launch_bounds__(kMbBlock) void k_mb_dev_add(uint32_t *__restrict__ set, uint32_t n,
                                                         uint32_t per_lane) {
  uint32_t h = lane_seed();
  for (uint32_t i = 0; i < per_lane; ++i) {
    h = h * kLcgMul + kLcgAdd;
    __hip_atomic_fetch_add(set + __umulhi(h, n), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kMbBlock) void k_mb_dev_min(unsigned long long *__restrict__ set,
                                                         uint32_t n, uint32_t per_lane) {
  uint32_t h = lane_seed();
  for (uint32_t i = 0; i < per_lane; ++i) {
    h = h * kLcgMul + kLcgAdd;
    const unsigned long long key = (static_cast<unsigned long long>(h) << 32) | (h >> 7);
    __hip_atomic_fetch_min(set + __umulhi(h, n), key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// LDS probes: 1024-lane workgroups (the count accumulate's shape), a 64 KiB
// table, and one word per workgroup written out so the work is kept.
constexpr int kMbLdsBlock = 1024;

__global__ __launch_bounds__(kMbLdsBlock) void k_mb_lds_add(uint32_t *__restrict__ out,
                                                            uint32_t per_lane) {
  __shared__ uint32_t tab[16384];
  for (int i = threadIdx.x; i < 16384; i += kMbLdsBlock) tab[i] = 0u;
  __syncthreads();
  uint32_t h = lane_seed();
  for (uint32_t i = 0; i < per_lane; ++i) {
    h = h * kLcgMul + kLcgAdd;
    atomicAdd(&tab[h >> 18], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = tab[h >> 18];
}

__global__ __launch_bounds__(kMbLdsBlock) void k_mb_lds_add64(unsigned long long *__restrict__ out,
                                                              uint32_t per_lane) {
  __shared__ unsigned long long tab[8192];
  for (int i = threadIdx.x; i < 8192; i += kMbLdsBlock) tab[i] = 0ull;
  __syncthreads();
  uint32_t h = lane_seed();
  for (uint32_t i = 0; i < per_lane; ++i) {
    h = h * kLcgMul + kLcgAdd;
    atomicAdd(&tab[h >> 19], static_cast<unsigned long long>(h | 1u));
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = tab[h >> 19];
}

__global__ __launch_bounds__(kMbLdsBlock) void k_mb_lds_min(unsigned long long *__restrict__ out,
                                                            uint32_t per_lane) {
  __shared__ unsigned long long tab[8192];
  for (int i = threadIdx.x; i < 8192; i += kMbLdsBlock) tab[i] = ~0ull;
  __syncthreads();
  uint32_t h = lane_seed();
  for (uint32_t i = 0; i < per_lane; ++i) {
    h = h * kLcgMul + kLcgAdd;
    atomicMin(&tab[h >> 19], (static_cast<unsigned long long>(h) << 32) | i);
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = tab[h >> 19];
}

__global__ __launch_bounds__(kMbBlock) void k_mb_philox(uint32_t *__restrict__ out,
                                                        uint32_t per_lane) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < per_lane; ++i) {
    const Block4 b = philox10(g, i, 0u, 0u, 0x12345678u, 0x9ABCDEF0u);
    acc ^= b.w0 ^ b.w1 ^ b.w2 ^ b.w3;
  }
  out[g] = acc;
}

// Groups of 2^LOG2G lanes; each group reads `per_group` runs of 2^LOG2G
// 16-byte vectors starting at random vectors of [0, n_start), four at a
// time; one word per lane is written so the loads are kept.
template <int LOG2G>
__global__ __launch_bounds__(kMbBlock) void k_mb_runs(const uint4 *__restrict__ buf,
                                                      uint32_t n_start, uint32_t per_group,
                                                      uint32_t *__restrict__ out) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = g & ((1u << LOG2G) - 1u);
  // the same sequence in every lane of a group
  uint32_t h = (g >> LOG2G) * 0x9E3779B9u + 0x7F4A7C15u;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < per_group; i += 4) {
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      h = h * kLcgMul + kLcgAdd;
      v[u] = buf[static_cast<size_t>(__umulhi(h, n_start)) + lane];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  out[g] = acc;
}

uint32_t per_lane_of(uint64_t ops, uint64_t lanes) {
  const uint64_t p = (ops + lanes - 1) / lanes;
  return static_cast<uint32_t>(p < 1 ? 1 : (p > 0xFFFFFFFFull ? 0xFFFFFFFFull : p));
}

}  // namespace

}  // namespace cfs

using namespace cfs;

extern "C" int cfs_microbench(int32_t kind, void *buf, size_t bytes, uint64_t ops,
                              uint64_t *done, void *stream) {
  clear_error();
  if (!buf || !done) return fail(CFS_E_INVALID, "buf/done is NULL");
  if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(CFS_E_INVALID, "buf must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t lanes = static_cast<uint64_t>(kMbGrid) * kMbBlock;
  switch (kind) {
    case CFS_MB_COPY: {
      const size_t n = bytes / 32;  // uint4 elements per half
      if (n == 0) return fail(CFS_E_INVALID, "copy needs at least 32 bytes");
      const uint4 *src = static_cast<const uint4 *>(buf);
      hipLaunchKernelGGL(k_mb_copy, dim3(kMbGrid), dim3(kMbBlock), 0, s, src,
                         static_cast<uint4 *>(buf) + n, n);
      *done = 2ull * n * sizeof(uint4);
      break;
    }
    case CFS_MB_DEV_ADD_U32:
    case CFS_MB_DEV_MIN_U64: {
      const size_t elem = kind == CFS_MB_DEV_ADD_U32 ? 4 : 8;
      const uint64_t n = bytes / elem;
      if (n == 0 || n > 0xFFFFFFFFull)
        return fail(CFS_E_INVALID, "working set must hold 1 .. 2^32 - 1 elements");
      const uint32_t pl = per_lane_of(ops, lanes);
      if (kind == CFS_MB_DEV_ADD_U32)
        hipLaunchKernelGGL(k_mb_dev_add, dim3(kMbGrid), dim3(kMbBlock), 0, s,
                           static_cast<uint32_t *>(buf), static_cast<uint32_t>(n), pl);
      else
        hipLaunchKernelGGL(k_mb_dev_min, dim3(kMbGrid), dim3(kMbBlock), 0, s,
                           static_cast<unsigned long long *>(buf), static_cast<uint32_t>(n), pl);
      *done = lanes * pl;
      break;
    }
    case CFS_MB_LDS_ADD_U32:
    case CFS_MB_LDS_ADD_U64:
    case CFS_MB_LDS_MIN_U64: {
      const uint32_t grid = 512;  // two 1024-lane workgroups per compute unit
      const size_t elem = kind == CFS_MB_LDS_ADD_U32 ? 4 : 8;
      if (bytes < grid * elem) return fail(CFS_E_INVALID, "buf must hold one word per workgroup");
      const uint32_t pl = per_lane_of(ops, static_cast<uint64_t>(grid) * kMbLdsBlock);
      if (kind == CFS_MB_LDS_ADD_U32)
        hipLaunchKernelGGL(k_mb_lds_add, dim3(grid), dim3(kMbLdsBlock), 0, s,
                           static_cast<uint32_t *>(buf), pl);
      else if (kind == CFS_MB_LDS_ADD_U64)
        hipLaunchKernelGGL(k_mb_lds_add64, dim3(grid), dim3(kMbLdsBlock), 0, s,
                           static_cast<unsigned long long *>(buf), pl);
      else
        hipLaunchKernelGGL(k_mb_lds_min, dim3(grid), dim3(kMbLdsBlock), 0, s,
                           static_cast<unsigned long long *>(buf), pl);
      *done = static_cast<uint64_t>(grid) * kMbLdsBlock * pl;
      break;
    }
    case CFS_MB_PHILOX: {
      if (bytes < lanes * 4) return fail(CFS_E_INVALID, "buf must hold one word per lane");
      const uint32_t pl = per_lane_of(ops, lanes);
      hipLaunchKernelGGL(k_mb_philox, dim3(kMbGrid), dim3(kMbBlock), 0, s,
                         static_cast<uint32_t *>(buf), pl);
      *done = lanes * pl;
      break;
    }
    case CFS_MB_RUNS_128:
    case CFS_MB_RUNS_512:
    case CFS_MB_RUNS_2048: {
      // buf = [lanes words written | the runs' buffer]
      const int lg = kind == CFS_MB_RUNS_128 ? 3 : (kind == CFS_MB_RUNS_512 ? 5 : 7);
      const uint32_t vec = 1u << lg;  // 16-byte vectors per run
      const size_t head = (lanes * 4 + 255) & ~static_cast<size_t>(255);
      if (bytes < head + (static_cast<size_t>(vec) << 4) * 2)
        return fail(CFS_E_INVALID, "buf must hold one word per lane and two runs");
      const uint64_t nv = (bytes - head) / 16;
      const uint64_t n_start = nv - vec + 1;
      if (n_start > 0xFFFFFFFFull) return fail(CFS_E_INVALID, "runs buffer above 64 GiB");
      const uint64_t groups = lanes >> lg;
      uint32_t pg = per_lane_of(ops, groups);
      pg = pg > 0xFFFFFFF0u ? 0xFFFFFFF0u : (pg + 3u) & ~3u;  // whole rounds of four
      const uint4 *runs = reinterpret_cast<const uint4 *>(static_cast<char *>(buf) + head);
      uint32_t *words = static_cast<uint32_t *>(buf);
      if (lg == 3)
        hipLaunchKernelGGL(k_mb_runs<3>, dim3(kMbGrid), dim3(kMbBlock), 0, s, runs,
                           static_cast<uint32_t>(n_start), pg, words);
      else if (lg == 5)
        hipLaunchKernelGGL(k_mb_runs<5>, dim3(kMbGrid), dim3(kMbBlock), 0, s, runs,
                           static_cast<uint32_t>(n_start), pg, words);
      else
        hipLaunchKernelGGL(k_mb_runs<7>, dim3(kMbGrid), dim3(kMbBlock), 0, s, runs,
                           static_cast<uint32_t>(n_start), pg, words);
      *done = groups * pg * (static_cast<uint64_t>(vec) << 4);  // bytes read
      break;
    }
    default:
      return fail(CFS_E_INVALID, "unknown microbenchmark kind %d", kind);
  }
  return device_status(hipGetLastError(), "cfs_microbench");
}
