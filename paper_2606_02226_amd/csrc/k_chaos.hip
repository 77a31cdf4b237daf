// k_chaos.hip -- the fused plain chaos game (Section 1 and Section 3 of the
// paper): per lane, draw the initial point, then for every iteration draw an
// index, apply that map, and after burn-in transform a copy and splat it.
//
// Layout: one point per lane, 256-lane workgroups; the map table and the
// selection thresholds are copied from kernel arguments into LDS once per
// workgroup and gathered by index.  Integer splats go straight to device
// memory with no-return atomics (u32 add; u64 min + u32 add for depth).
#include "cfs_device.hpp"
#include "cfs_host.hpp"

namespace cfs {

constexpr int kChaosBlock = 256;

template <typename real, int DIM, int FINAL, bool EQUAL, bool DEPTH>
__global__ __launch_bounds__(kChaosBlock) void k_chaos(MapTable<DIM> mt, Window win,
                                                       RunArgs ra, FinalArgs fa, void *img,
                                                       uint32_t *density, float near_plane,
                                                       Outputs out) {
  __shared__ real table[kMaxMaps * RowStride<real, DIM>::value];
  __shared__ uint32_t th[kMaxMaps];
  load_table<real, DIM>(mt, table, th);
  __syncthreads();

  const uint32_t n = blockIdx.x * kChaosBlock + threadIdx.x;
  if (n >= ra.n_points) return;
  const uint32_t pid = ra.point_offset + n;
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const size_t plane = static_cast<size_t>(win.width) * static_cast<size_t>(win.height);

  real p[DIM];
  initial_point<real, DIM>(pid, ra.instance, ra.k0, ra.k1, p);
  int k = 0;
  uint32_t dropped = 0;

  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, t0 >> 2, ra.instance, 0u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const uint32_t u = word_of(blk, j);
      if constexpr (EQUAL)
        k = select_equal(u, static_cast<uint32_t>(mt.n_maps));
      else
        k = select_table(u, th, mt.n_search, mt.top_step);
      if (out.indices) out.indices[static_cast<size_t>(n) * T + (t - 1)] = static_cast<uint8_t>(k);
      apply_map<real, DIM>(table, k, p);
      if (t > B) {
        real q[2];
        real depth = static_cast<real>(0);
        final_transform<real, FINAL, DIM>(fa.p, p, q, &depth);
        int ix;
        int pix = bin_pixel<real>(q, win, &ix);
        if constexpr (DEPTH) {
          if (!(depth > static_cast<real>(near_plane))) pix = -1;
        }
        if (pix < 0) {
          ++dropped;
        } else if constexpr (DEPTH) {
          const float zf = static_cast<float>(depth);
          const unsigned long long key =
              (static_cast<unsigned long long>(__float_as_uint(zf)) << 32) |
              static_cast<unsigned long long>(k);
          atomicMin(static_cast<unsigned long long *>(img) + pix, key);
          __hip_atomic_fetch_add(density + pix, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          const size_t at = (win.by_index ? static_cast<size_t>(k) * plane : 0) +
                            static_cast<size_t>(pix);
          __hip_atomic_fetch_add(static_cast<uint32_t *>(img) + at, 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }

  if (out.final_points) {
    real *fp = static_cast<real *>(out.final_points) + static_cast<size_t>(n) * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) fp[c] = p[c];
  }
  if (out.last_index) out.last_index[n] = static_cast<uint8_t>(k);
  if (out.dropped && dropped)
    __hip_atomic_fetch_add(out.dropped, static_cast<unsigned long long>(dropped),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename real, int DIM, int FINAL, bool EQUAL, bool DEPTH>
static hipError_t launch_typed(const ChaosJob &j, hipStream_t s) {
  const uint32_t blocks = (j.ra.n_points + kChaosBlock - 1) / kChaosBlock;
  const MapTable<DIM> &mt = [&]() -> const MapTable<DIM> & {
    if constexpr (DIM == 2) return j.mt2; else return j.mt3;
  }();
  hipLaunchKernelGGL((k_chaos<real, DIM, FINAL, EQUAL, DEPTH>), dim3(blocks), dim3(kChaosBlock),
                     0, s, mt, j.win, j.ra, j.fa, j.img, j.density, j.near_plane, j.out);
  return hipGetLastError();
}

template <typename real, int DIM, int FINAL, bool DEPTH>
static hipError_t launch_sel(const ChaosJob &j, hipStream_t s) {
  return j.equal ? launch_typed<real, DIM, FINAL, true, DEPTH>(j, s)
                 : launch_typed<real, DIM, FINAL, false, DEPTH>(j, s);
}

template <typename real>
static hipError_t launch_real(const ChaosJob &j, hipStream_t s) {
  if (j.dim == 2) {
    switch (j.final_kind) {
      case kFinalSwirl: return launch_sel<real, 2, kFinalSwirl, false>(j, s);
      case kFinalStretch: return launch_sel<real, 2, kFinalStretch, false>(j, s);
      default: return launch_sel<real, 2, kFinalIdentity, false>(j, s);
    }
  }
  if (j.depth) return launch_sel<real, 3, kFinalTwistCamera, true>(j, s);
  return launch_sel<real, 3, kFinalIdentity, false>(j, s);
}

hipError_t launch_chaos(const ChaosJob &job, hipStream_t stream) {
  if (job.ra.n_points == 0) return hipSuccess;
  return job.precision == 1 ? launch_real<double>(job, stream) : launch_real<float>(job, stream);
}

}  // namespace cfs
