// k_scene.hip -- several objects from one primitive (Section 3, multiple
// objects from a single primitive; fig. "space").
//
// Each lane iterates one point of a 2D primitive exactly like the plain
// chaos game.  After burn-in, every step repositions a copy of the point once
// per object (the object's transform, then its placement, then -- for
// duplicated objects -- the scale and offset of the copy its random stream
// picks) and splats each copy into the object's channel.  Nothing but the
// image lives in device memory; copy positions come from Philox on the fly.
//
// Two splat paths, as for the plain count image: direct device atomics, or
// the binned path (LDS tile sort per chunk of kBinSlots records per lane,
// then the per-tile accumulate), which is bit-identical.
#include "cfs_binned.hpp"
#include "cfs_host.hpp"

namespace cfs {

namespace {

// Placement of copy c of object o: scale and offset from Philox block
// (c, o, instance, 3).
template <typename real>
__device__ __forceinline__ void copy_placement(const SceneObject &ob, uint32_t c, uint32_t o,
                                               uint32_t instance, uint32_t k0, uint32_t k1,
                                               real *sc, real *off0, real *off1) {
  const Block4 w = philox10(c, o, instance, 3u, k0, k1);
  const real e0 = static_cast<real>(w.w0 >> 8) * static_cast<real>(0x1p-24);
  const real e1 = static_cast<real>(w.w1 >> 8) * static_cast<real>(0x1p-24);
  const real e2 = static_cast<real>(w.w2 >> 8) * static_cast<real>(0x1p-24);
  *sc = static_cast<real>(ob.scale_lo) + static_cast<real>(ob.scale_span) * e2;
  *off0 = static_cast<real>(ob.copy_lo[0]) + static_cast<real>(ob.copy_span[0]) * e0;
  *off1 = static_cast<real>(ob.copy_lo[1]) + static_cast<real>(ob.copy_span[1]) * e1;
}

// Every workgroup fills the LDS placement rows of the objects that have them
// (kSceneCopyTable rows of scale, offset x, offset y); callers sync after.
template <typename real>
__device__ inline void load_copy_table(const SceneArgs &sc, const RunArgs &ra, real *ctab) {
  for (int o = 0; o < sc.n_obj; ++o) {
    const SceneObject &ob = sc.obj[o];
    if (ob.tab_base < 0) continue;
    for (uint32_t c = threadIdx.x; c < ob.n_copies; c += blockDim.x) {
      real *row = ctab + 3 * (static_cast<uint32_t>(ob.tab_base) + c);
      copy_placement<real>(ob, c, static_cast<uint32_t>(o), ra.instance, ra.k0, ra.k1, row,
                           row + 1, row + 2);
    }
  }
}

// The object transform (a wave-uniform branch on the kind), then placement
// and duplication.  `cu` is the copy draw of this iteration; the copy's
// placement comes from the LDS rows when the object has them.
template <typename real>
__device__ __forceinline__ void object_copy(const SceneObject &ob, uint32_t o, const real p[2],
                                            uint32_t cu, uint32_t instance, uint32_t k0,
                                            uint32_t k1, const real *ctab, real q[2]) {
  real g[2], dz;
  switch (ob.kind) {
    case kFinalSwirl: final_transform<real, kFinalSwirl, 2>(ob.fp, p, g, &dz); break;
    case kFinalStretch: final_transform<real, kFinalStretch, 2>(ob.fp, p, g, &dz); break;
    case kFinalRing: final_transform<real, kFinalRing, 2>(ob.fp, p, g, &dz); break;
    default: g[0] = p[0]; g[1] = p[1]; break;
  }
  q[0] = static_cast<real>(ob.place[0]) * g[0] + static_cast<real>(ob.place[1]) * g[1] +
         static_cast<real>(ob.place[4]);
  q[1] = static_cast<real>(ob.place[2]) * g[0] + static_cast<real>(ob.place[3]) * g[1] +
         static_cast<real>(ob.place[5]);
  if (ob.n_copies > 1) {
    const uint32_t c = __umulhi((2u * o + 1u) * cu, ob.n_copies);
    real sc, off0, off1;
    if (ob.tab_base >= 0) {
      const real *row = ctab + 3 * (static_cast<uint32_t>(ob.tab_base) + c);
      sc = row[0];
      off0 = row[1];
      off1 = row[2];
    } else {
      copy_placement<real>(ob, c, o, instance, k0, k1, &sc, &off0, &off1);
    }
    q[0] = sc * q[0] + off0;
    q[1] = sc * q[1] + off1;
  }
}

constexpr int kSceneBlock = 256;

template <typename real, int SEL>
__global__ __launch_bounds__(kSceneBlock) void k_scene(MapTable<2> mt, Window win, RunArgs ra,
                                                       SceneArgs sc, uint32_t *img,
                                                       unsigned long long *dropped_out) {
  __shared__ real table[kMaxMaps * RowStride<real, 2>::value];
  __shared__ uint32_t th[kThWords];
  __shared__ real ctab[3 * kSceneCopyTable];
  load_table<real, 2>(mt, table, th);
  load_copy_table<real>(sc, ra, ctab);
  __syncthreads();
  const uint32_t n = blockIdx.x * kSceneBlock + threadIdx.x;
  if (n >= ra.n_points) return;
  const uint32_t pid = ra.point_offset + n;
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const uint32_t plane = static_cast<uint32_t>(win.width) * static_cast<uint32_t>(win.height);
  real p[2];
  initial_point<real, 2>(pid, ra.instance, ra.k0, ra.k1, p);
  uint32_t dropped = 0;
  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, t0 >> 2, ra.instance, 0u, ra.k0, ra.k1);
    Block4 cblk{0u, 0u, 0u, 0u};
    if (sc.any_copies && t0 + 4 > B) cblk = philox10(pid, t0 >> 2, ra.instance, 2u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const int k = select_index<SEL>(word_of(blk, j), th, mt.n_maps, mt.n_search);
      apply_map<real, 2>(table, k, p, mt.flags);
      if (t <= B) continue;
      const uint32_t cu = word_of(cblk, j);
      for (int o = 0; o < sc.n_obj; ++o) {
        real q[2];
        object_copy<real>(sc.obj[o], static_cast<uint32_t>(o), p, cu, ra.instance, ra.k0, ra.k1,
                          ctab, q);
        int ix;
        const int pix = bin_pixel<real>(q, win, &ix);
        if (pix < 0) {
          ++dropped;
        } else {
          __hip_atomic_fetch_add(img + static_cast<uint32_t>(sc.obj[o].channel) * plane +
                                     static_cast<uint32_t>(pix),
                                 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
  if (dropped_out && dropped)
    __hip_atomic_fetch_add(dropped_out, static_cast<unsigned long long>(dropped), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Binned: every lane stages n_obj records per step after burn-in; a full
// stage of kBinSlots records per lane is flushed (the flush is block-wide,
// and every lane reaches it after the same number of records).  Four waves
// per SIMD (two workgroups per CU) are asked for: the FP64 object transforms
// would otherwise take 160 VGPRs and leave one workgroup per CU (3.65 ms
// instead of 4.28 ms per 1920x1080 frame, with a few spilled registers).
template <typename real, int SEL>
__global__ __launch_bounds__(kBinBlock, 4) void k_scene_binned(MapTable<2> mt, Window win,
                                                            RunArgs ra, SceneArgs sc, BinArgs ba,
                                                            unsigned long long *dropped_out) {
  __shared__ real table[kMaxMaps * RowStride<real, 2>::value];
  __shared__ uint32_t th[kThWords];
  __shared__ uint32_t stage[kChunkCap];
  __shared__ uint32_t cnt[kMaxTiles];
  __shared__ uint32_t wsum[kWaves + 1];
  __shared__ real ctab[3 * kSceneCopyTable];
  load_table<real, 2>(mt, table, th);
  load_copy_table<real>(sc, ra, ctab);
  for (uint32_t t = threadIdx.x; t < ba.n_tiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();

  const int tid = threadIdx.x;
  const uint32_t n = blockIdx.x * kBinBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const uint32_t plane = static_cast<uint32_t>(win.width) * static_cast<uint32_t>(win.height);
  real p[2];
  initial_point<real, 2>(pid, ra.instance, ra.k0, ra.k1, p);
  uint32_t dropped = 0;
  int slot = 0;
  uint32_t chunk = blockIdx.x * ba.flushes;
  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, t0 >> 2, ra.instance, 0u, ra.k0, ra.k1);
    Block4 cblk{0u, 0u, 0u, 0u};
    if (sc.any_copies && t0 + 4 > B) cblk = philox10(pid, t0 >> 2, ra.instance, 2u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const int k = select_index<SEL>(word_of(blk, j), th, mt.n_maps, mt.n_search);
      apply_map<real, 2>(table, k, p, mt.flags);
      if (t <= B) continue;
      const uint32_t cu = word_of(cblk, j);
      for (int o = 0; o < sc.n_obj; ++o) {
        uint32_t e = kInvalid;
        if (active) {
          real q[2];
          object_copy<real>(sc.obj[o], static_cast<uint32_t>(o), p, cu, ra.instance, ra.k0, ra.k1,
                            ctab, q);
          int ix;
          const int pix = bin_pixel<real>(q, win, &ix);
          if (pix >= 0)
            e = static_cast<uint32_t>(sc.obj[o].channel) * plane + static_cast<uint32_t>(pix);
          else
            ++dropped;
        }
        stage[slot * kBinBlock + tid] = e;
        if (e != kInvalid) atomicAdd(&cnt[e >> kTileBits], 1u);
        if (++slot == kBinSlots) {
          flush_chunk(stage, cnt, wsum, slot, chunk, ba);
          slot = 0;
          ++chunk;
        }
      }
    }
  }
  if (slot > 0) flush_chunk(stage, cnt, wsum, slot, chunk, ba);
  if (active && dropped_out && dropped)
    __hip_atomic_fetch_add(dropped_out, static_cast<unsigned long long>(dropped), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename real, int SEL>
hipError_t launch_scene_typed(const SceneJob &j, hipStream_t s) {
  if (!j.binned) {
    const uint32_t blocks = (j.ra.n_points + kSceneBlock - 1) / kSceneBlock;
    hipLaunchKernelGGL((k_scene<real, SEL>), dim3(blocks), dim3(kSceneBlock), 0, s, j.mt, j.win,
                       j.ra, j.sc, j.img, j.dropped);
    return hipGetLastError();
  }
  const uint32_t blocks = (j.ra.n_points + kBinBlock - 1) / kBinBlock;
  hipLaunchKernelGGL((k_scene_binned<real, SEL>), dim3(blocks), dim3(kBinBlock), 0, s, j.mt, j.win,
                     j.ra, j.sc, j.ba, j.dropped);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || j.ba.n_chunks == 0) return e;
  return launch_count_accumulate(j.ba, j.img, s);
}

template <typename real>
hipError_t launch_scene_real(const SceneJob &j, hipStream_t s) {
  return j.equal ? launch_scene_typed<real, kSelEqual>(j, s)
                 : launch_scene_typed<real, kSelTable>(j, s);
}

}  // namespace

hipError_t launch_scene(const SceneJob &job, hipStream_t stream) {
  if (job.ra.n_points == 0) return hipSuccess;
  return job.precision == 1 ? launch_scene_real<double>(job, stream)
                            : launch_scene_real<float>(job, stream);
}

}  // namespace cfs
