// cfs_direct.hpp -- the chaos game of one point with the direct splat, shared
// by the plain direct kernel and the batched persistent kernel.
#pragma once

#include "cfs_device.hpp"

namespace cfs {

// The chaos game of point n of a run with the direct splat (one device
// atomic per splat).  table/th hold the map table in LDS.
// GENERAL as for chaos_binned_block.
template <typename real, int DIM, int FINAL, int SEL, bool DEPTH, bool GENERAL = true>
__device__ void chaos_direct_point(const real *table, const uint32_t *th, int n_maps, int n_search,
                                   int flags, const Window &win, const RunArgs &ra,
                                   const float *fparams, void *img, uint32_t *density,
                                   float near_plane, const Outputs &out, uint32_t n) {
  if constexpr (!GENERAL) flags = 0;
  if (n >= ra.n_points) return;
  const uint32_t pid = ra.point_offset + n;
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const size_t plane = static_cast<size_t>(win.width) * static_cast<size_t>(win.height);

  // continued runs take the general variant, as in chaos_binned_block
  real p[DIM];
  if constexpr (GENERAL)
    start_point<real, DIM>(ra, pid, n, true, out.final_points, p);
  else
    initial_point<real, DIM>(pid, ra.instance, ra.k0, ra.k1, p);
  const uint32_t blk0 = GENERAL ? ra.iter_block : 0u;
  int k = 0;
  uint32_t dropped = 0;

  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, (t0 >> 2) + blk0, ra.instance, 0u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const uint32_t u = word_of(blk, j);
      k = select_index<SEL>(u, th, n_maps, n_search);
      if (out.indices) out.indices[static_cast<size_t>(n) * T + (t - 1)] = static_cast<uint8_t>(k);
      apply_map<real, DIM>(table, k, p, flags);
      if constexpr (DIM == 2 && FINAL != kFinalIdentity) {
        if (flags & kFlagReuse) {
          real g[2], dz;
          final_transform<real, FINAL, DIM>(fparams, p, g, &dz);
          p[0] = g[0];
          p[1] = g[1];
        }
      }
      if (t > B) {
        real q[2];
        real depth = static_cast<real>(0);
        if constexpr (DIM == 2 && FINAL != kFinalIdentity) {
          if (flags & kFlagReuse) {
            q[0] = p[0];
            q[1] = p[1];
          } else {
            final_transform<real, FINAL, DIM>(fparams, p, q, &depth);
          }
        } else {
          final_transform<real, FINAL, DIM>(fparams, p, q, &depth);
        }
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

}  // namespace cfs
