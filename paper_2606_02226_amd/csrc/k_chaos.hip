// k_chaos.hip -- the fused plain chaos game (Section 1 and Section 3 of the
// paper): per lane, draw the initial point, then for every iteration draw an
// index, apply that map, and after burn-in transform a copy and splat it.
//
// Layout: one point per lane, 256-lane workgroups; the map table and the
// selection thresholds are copied from kernel arguments into LDS once per
// workgroup and gathered by index.  Integer splats go straight to device
// memory with no-return atomics (u32 add; u64 min + u32 add for depth).
#include "cfs_direct.hpp"
#include "cfs_host.hpp"

namespace cfs {

constexpr int kChaosBlock = 256;

template <typename real, int DIM, int FINAL, bool EQUAL, bool DEPTH, bool GENERAL>
__global__ __launch_bounds__(kChaosBlock) void k_chaos(MapTable<DIM> mt, Window win,
                                                       RunArgs ra, FinalArgs fa, void *img,
                                                       uint32_t *density, float near_plane,
                                                       Outputs out) {
  __shared__ real table[kMaxMaps * RowStride<real, DIM>::value];
  __shared__ uint32_t th[kThWords];
  load_table<real, DIM>(mt, table, th);
  __syncthreads();
  chaos_direct_point<real, DIM, FINAL, EQUAL, DEPTH, GENERAL>(
      table, th, mt.n_maps, mt.n_search, mt.flags, win, ra, fa.p, img, density,
      near_plane, out, blockIdx.x * kChaosBlock + threadIdx.x);
}

template <typename real, int DIM, int FINAL, bool EQUAL, bool DEPTH>
static hipError_t launch_typed(const ChaosJob &j, hipStream_t s) {
  const uint32_t blocks = (j.ra.n_points + kChaosBlock - 1) / kChaosBlock;
  const MapTable<DIM> &mt = [&]() -> const MapTable<DIM> & {
    if constexpr (DIM == 2) return j.mt2; else return j.mt3;
  }();
  // circle maps, reuse composition (2D only) and continued runs take the
  // general variant
  if (mt.flags != 0 || j.ra.iter_block != 0)
    hipLaunchKernelGGL((k_chaos<real, DIM, FINAL, EQUAL, DEPTH, true>), dim3(blocks),
                       dim3(kChaosBlock), 0, s, mt, j.win, j.ra, j.fa, j.img, j.density,
                       j.near_plane, j.out);
  else
    hipLaunchKernelGGL((k_chaos<real, DIM, FINAL, EQUAL, DEPTH, false>), dim3(blocks),
                       dim3(kChaosBlock), 0, s, mt, j.win, j.ra, j.fa, j.img, j.density,
                       j.near_plane, j.out);
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
      case kFinalRing: return launch_sel<real, 2, kFinalRing, false>(j, s);
      default: return launch_sel<real, 2, kFinalIdentity, false>(j, s);
    }
  }
  if (j.depth) return launch_sel<real, 3, kFinalTwistCamera, true>(j, s);
  return launch_sel<real, 3, kFinalIdentity, false>(j, s);
}

hipError_t launch_chaos(const ChaosJob &job, hipStream_t stream) {
  hipError_t e = hipSuccess;
  mark_phase(job.ev, 0, stream);
  if (job.ra.n_points != 0)
    e = job.precision == 1 ? launch_real<double>(job, stream) : launch_real<float>(job, stream);
  // the direct path has no transpose or accumulate phase
  for (int i = 1; i < kPhaseEvents; ++i) mark_phase(job.ev, i, stream);
  return e;
}

}  // namespace cfs
