// k_binned.hip -- chaos game with a binned integer splat.
//
// Device-wide atomics on MI355X sustain about 27 G random updates/s no matter
// how small the image is, while LDS atomics are an order of magnitude faster.
// The splat (Section 1: each iterate colours its pixel; Section 4: density
// estimation needs atomics) is therefore split in two kernels:
//   1. k_chaos_binned runs the chaos game exactly like the direct kernel and
//      collects kBinSlots splats per lane in LDS.  Each full stage (a chunk)
//      is sorted by image tile with LDS atomics and written out contiguously
//      as 16-bit in-tile offsets, plus one column of a [tile][chunk] table of
//      run starts.  No device-wide atomics.
//   2. k_tile_accumulate gives each image tile one workgroup, counts the
//      tile's runs of every chunk in an LDS histogram and adds it into the
//      image.  Integer sums are order-independent, so the image is
//      bit-identical to the direct path.
#include "cfs_device.hpp"
#include "cfs_host.hpp"

namespace cfs {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kWaves = kBinBlock / 64;

// Exclusive prefix sum of a[0..n) in place (n <= 2 * kBinBlock), returns the
// total.  Every thread of the block must call it.
__device__ uint32_t block_exclusive_scan(uint32_t *a, uint32_t n, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t i0 = 2u * tid, i1 = i0 + 1u;
  const uint32_t v0 = i0 < n ? a[i0] : 0u;
  const uint32_t v1 = i1 < n ? a[i1] : 0u;
  const uint32_t s = v0 + v1;
  uint32_t incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    const uint32_t x = lane < kWaves ? wsum[lane] : 0u;
    uint32_t xi = x;
#pragma unroll
    for (int d = 1; d < kWaves; d <<= 1) {
      const uint32_t y = __shfl_up(xi, d, 64);
      if (lane >= d) xi += y;
    }
    if (lane < kWaves) wsum[lane] = xi - x;
    if (lane == kWaves - 1) wsum[kWaves] = xi;
  }
  __syncthreads();
  const uint32_t excl = wsum[w] + incl - s;
  if (i0 < n) a[i0] = excl;
  if (i1 < n) a[i1] = excl + v0;
  const uint32_t total = wsum[kWaves];
  __syncthreads();
  return total;
}

// Sort the stage of one chunk by tile and write it out (all threads call it).
// cnt[t] holds the number of stage records of tile t on entry and is zero on
// return.
__device__ void flush_chunk(uint32_t *stage, uint32_t *cnt, uint32_t *wsum, int used_slots,
                            uint32_t chunk, const BinArgs &ba) {
  __syncthreads();
  const int tid = threadIdx.x;
  const uint32_t total = block_exclusive_scan(cnt, ba.n_tiles, wsum);
  const uint32_t base = chunk * kChunkCap;
  for (uint32_t t = tid; t <= ba.n_tiles; t += kBinBlock)
    ba.tile_start[static_cast<size_t>(t) * ba.n_chunks + chunk] =
        base + (t < ba.n_tiles ? cnt[t] : total);
  uint32_t e[kBinSlots];
#pragma unroll
  for (int i = 0; i < kBinSlots; ++i) e[i] = i < used_slots ? stage[i * kBinBlock + tid] : kInvalid;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBinSlots; ++i) {
    if (e[i] != kInvalid) {
      const uint32_t pos = atomicAdd(&cnt[e[i] >> kTileBits], 1u);
      stage[pos] = e[i];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < total; i += kBinBlock)
    ba.records[static_cast<size_t>(base) + i] = static_cast<uint16_t>(stage[i] & (kTileElems - 1));
  for (uint32_t t = tid; t < ba.n_tiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();
}

template <typename real, int DIM, int FINAL, bool EQUAL>
__global__ __launch_bounds__(kBinBlock) void k_chaos_binned(MapTable<DIM> mt, Window win,
                                                            RunArgs ra, FinalArgs fa, BinArgs ba,
                                                            Outputs out) {
  __shared__ real table[kMaxMaps * RowStride<real, DIM>::value];
  __shared__ uint32_t th[kMaxMaps];
  __shared__ uint32_t stage[kChunkCap];
  __shared__ uint32_t cnt[kMaxTiles];
  __shared__ uint32_t wsum[kWaves + 1];
  const int tid = threadIdx.x;
  load_table<real, DIM>(mt, table, th);
  for (uint32_t t = tid; t < ba.n_tiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();

  const uint32_t n = blockIdx.x * kBinBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const uint32_t plane = static_cast<uint32_t>(win.width) * static_cast<uint32_t>(win.height);

  real p[DIM];
  initial_point<real, DIM>(pid, ra.instance, ra.k0, ra.k1, p);
  int k = 0;
  uint32_t dropped = 0;
  int slot = 0;
  uint32_t chunk = blockIdx.x * ba.flushes;

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
      if (active && out.indices)
        out.indices[static_cast<size_t>(n) * T + (t - 1)] = static_cast<uint8_t>(k);
      apply_map<real, DIM>(table, k, p);
      if (t > B) {
        uint32_t e = kInvalid;
        if (active) {
          real q[2];
          real depth = static_cast<real>(0);
          final_transform<real, FINAL, DIM>(fa.p, p, q, &depth);
          int ix;
          const int pix = bin_pixel<real>(q, win, &ix);
          if (pix >= 0)
            e = (win.by_index ? static_cast<uint32_t>(k) * plane : 0u) + static_cast<uint32_t>(pix);
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

  if (!active) return;
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

// One workgroup per image tile: LDS histogram of the tile's records from every
// chunk, then add it into the image (the workgroup owns the tile).
__global__ __launch_bounds__(kAccBlock) void k_tile_accumulate(const uint16_t *__restrict__ rec,
                                                               const uint32_t *__restrict__ tile_start,
                                                               uint32_t n_chunks, uint32_t elems,
                                                               uint32_t *__restrict__ img) {
  __shared__ uint32_t tile[kTileElems];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t t = blockIdx.x;
  for (uint32_t i = tid; i < kTileElems; i += kAccBlock) tile[i] = 0u;
  __syncthreads();
  const uint32_t *row0 = tile_start + static_cast<size_t>(t) * n_chunks;
  const uint32_t *row1 = row0 + n_chunks;
  constexpr int kAccWaves = kAccBlock / 64;
  for (uint32_t cb = static_cast<uint32_t>(w) * 64u; cb < n_chunks; cb += kAccWaves * 64u) {
    const uint32_t c = cb + lane;
    const uint32_t s = c < n_chunks ? row0[c] : 0u;
    const uint32_t e = c < n_chunks ? row1[c] : 0u;
    // enumerate 64-record slabs of the 64 runs held by the lanes
    const uint32_t ns = (e - s + 63u) >> 6;
    uint32_t incl = ns;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const uint32_t excl = incl - ns;
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    for (uint32_t g0 = 0; g0 < total; g0 += 8) {
      uint32_t r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        r[u] = 0xFFFFu;
        const uint32_t g = g0 + u;
        if (g < total) {
          const unsigned long long m = __ballot(incl <= g);
          const int j = __popcll(m);
          const uint32_t sj = __builtin_amdgcn_readlane(s, j);
          const uint32_t ej = __builtin_amdgcn_readlane(e, j);
          const uint32_t xj = __builtin_amdgcn_readlane(excl, j);
          const uint32_t idx = sj + (g - xj) * 64u + static_cast<uint32_t>(lane);
          if (idx < ej) r[u] = rec[idx];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (r[u] != 0xFFFFu) atomicAdd(&tile[r[u]], 1u);
    }
  }
  __syncthreads();
  const uint32_t base = t * kTileElems;
  const uint32_t len = min(kTileElems, elems - base);
  for (uint32_t i = tid; i < len; i += kAccBlock) {
    const uint32_t v = tile[i];
    if (v) img[base + i] += v;
  }
}

BinPlan bin_plan(uint32_t points, uint32_t n_iters, uint32_t burn_in, uint32_t elems) {
  BinPlan bp{};
  bp.blocks = (points + kBinBlock - 1) / kBinBlock;
  bp.flushes = (n_iters - burn_in + kBinSlots - 1) / kBinSlots;
  bp.n_chunks = bp.blocks * bp.flushes;
  bp.n_tiles = (elems + kTileElems - 1) / kTileElems;
  bp.elems = elems;
  bp.records_bytes = static_cast<size_t>(bp.n_chunks) * kChunkCap * sizeof(uint16_t);
  bp.table_bytes = static_cast<size_t>(bp.n_tiles + 1) * bp.n_chunks * sizeof(uint32_t);
  return bp;
}

template <typename real, int DIM, int FINAL, bool EQUAL>
static hipError_t launch_binned_typed(const ChaosJob &j, hipStream_t s) {
  const MapTable<DIM> &mt = [&]() -> const MapTable<DIM> & {
    if constexpr (DIM == 2) return j.mt2; else return j.mt3;
  }();
  const uint32_t blocks = (j.ra.n_points + kBinBlock - 1) / kBinBlock;
  hipLaunchKernelGGL((k_chaos_binned<real, DIM, FINAL, EQUAL>), dim3(blocks), dim3(kBinBlock), 0,
                     s, mt, j.win, j.ra, j.fa, j.ba, j.out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || j.ba.n_chunks == 0) return e;
  hipLaunchKernelGGL(k_tile_accumulate, dim3(j.ba.n_tiles), dim3(kAccBlock), 0, s, j.ba.records,
                     j.ba.tile_start, j.ba.n_chunks, j.ba.elems, static_cast<uint32_t *>(j.img));
  return hipGetLastError();
}

template <typename real, int DIM, int FINAL>
static hipError_t launch_binned_sel(const ChaosJob &j, hipStream_t s) {
  return j.equal ? launch_binned_typed<real, DIM, FINAL, true>(j, s)
                 : launch_binned_typed<real, DIM, FINAL, false>(j, s);
}

template <typename real>
static hipError_t launch_binned_real(const ChaosJob &j, hipStream_t s) {
  if (j.dim == 3) return launch_binned_sel<real, 3, kFinalIdentity>(j, s);
  switch (j.final_kind) {
    case kFinalSwirl: return launch_binned_sel<real, 2, kFinalSwirl>(j, s);
    case kFinalStretch: return launch_binned_sel<real, 2, kFinalStretch>(j, s);
    default: return launch_binned_sel<real, 2, kFinalIdentity>(j, s);
  }
}

hipError_t launch_chaos_binned(const ChaosJob &job, hipStream_t stream) {
  if (job.ra.n_points == 0) return hipSuccess;
  return job.precision == 1 ? launch_binned_real<double>(job, stream)
                            : launch_binned_real<float>(job, stream);
}

}  // namespace cfs
