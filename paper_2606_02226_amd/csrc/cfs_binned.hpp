// cfs_binned.hpp -- device functions of the binned integer splat, shared by
// the plain binned kernels and the batched persistent kernels (so a batched
// instance runs exactly the code of a plain run).
#pragma once

#include "cfs_device.hpp"

namespace cfs {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kWaves = kBinBlock / 64;
constexpr int kDWaves = kDBlock / 64;

// Exclusive prefix sum of a[0..n) in place (n <= kMaxTiles), returns the
// total.  Thread i of the BLOCK threads owns kMaxTiles / BLOCK consecutive
// entries.  Every thread of the workgroup must call it; wsum holds
// BLOCK / 64 + 1 words.
template <int BLOCK = kBinBlock>
__device__ inline uint32_t block_exclusive_scan(uint32_t *a, uint32_t n, uint32_t *wsum) {
  constexpr int kPer = (kMaxTiles + BLOCK - 1) / BLOCK;
  constexpr int kW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t i0 = static_cast<uint32_t>(tid) * kPer;
  uint32_t v[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = i0 + q < n ? a[i0 + q] : 0u;
    s += v[q];
  }
  uint32_t incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    const uint32_t x = lane < kW ? wsum[lane] : 0u;
    uint32_t xi = x;
#pragma unroll
    for (int d = 1; d < kW; d <<= 1) {
      const uint32_t y = __shfl_up(xi, d, 64);
      if (lane >= d) xi += y;
    }
    if (lane < kW) wsum[lane] = xi - x;
    if (lane == kW - 1) wsum[kW] = xi;
  }
  __syncthreads();
  uint32_t run = wsum[w] + incl - s;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (i0 + q < n) a[i0 + q] = run;
    run += v[q];
  }
  const uint32_t total = wsum[kW];
  __syncthreads();
  return total;
}

// Sort the stage of one chunk by tile and write it out (all threads call it).
// On entry cnt[t] holds the number of stage records of tile t (counted as
// they were staged); the counts are scanned into tile starts, each record
// takes its slot from an LDS cursor per tile, and the sorted stage is written
// out.  cnt[] is zero on return.
__device__ inline void flush_chunk(uint32_t *stage, uint32_t *cnt, uint32_t *wsum, int used_slots,
                                   uint32_t chunk, const BinArgs &ba) {
  __syncthreads();
  const int tid = threadIdx.x;
  const uint32_t total = block_exclusive_scan(cnt, ba.n_tiles, wsum);
  const uint32_t base = chunk * kChunkCap;
  // run starts relative to the chunk (at most kChunkCap: 16 bits)
  uint16_t *row = ba.chunk_start + static_cast<size_t>(chunk) * (ba.n_tiles + 1);
  for (uint32_t t = tid; t <= ba.n_tiles; t += kBinBlock)
    row[t] = static_cast<uint16_t>(t < ba.n_tiles ? cnt[t] : total);
  uint32_t e[kBinSlots];
#pragma unroll
  for (int i = 0; i < kBinSlots; ++i) e[i] = i < used_slots ? stage[i * kBinBlock + tid] : kInvalid;
  __syncthreads();  // all stage entries read and table column written
#pragma unroll
  for (int i = 0; i < kBinSlots; ++i)
    if (e[i] != kInvalid) stage[atomicAdd(&cnt[e[i] >> kTileBits], 1u)] = e[i];
  __syncthreads();
  // two 16-bit records per 32-bit store (chunk bases are even)
  uint32_t *out32 = reinterpret_cast<uint32_t *>(ba.records + base);
  for (uint32_t i = tid; 2 * i < total; i += kBinBlock) {
    const uint32_t lo = stage[2 * i] & (kTileElems - 1);
    const uint32_t hi = 2 * i + 1 < total ? (stage[2 * i + 1] & (kTileElems - 1)) : 0xFFFFu;
    out32[i] = lo | (hi << 16);
  }
  for (uint32_t t = tid; t < ba.n_tiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();
}

// One block of kBinBlock points (block index `block` of the run): the chaos
// game of each lane's point with the binned splat.  table/th hold the map
// table in LDS; cnt[0 .. n_tiles) must be zero on entry and is zero on exit.
// Every thread of the workgroup calls it (it holds barriers).  GENERAL
// compiles the circle-map and reuse branches (`flags`) and continued runs
// (RunArgs::iter_block); without it they are compiled out, which keeps the
// affine copy-transform loop at its register count.
// LIN != kLinGeneral (with !GENERAL): the maps share one linear part `A` and
// `table` is the translations-only table.
template <typename real, int DIM, int FINAL, int SEL, bool GENERAL = true, int LIN = kLinGeneral>
__device__ void chaos_binned_block(const real *table, const uint32_t *th, int n_maps, int n_search,
                                   int flags, const Window &win, const RunArgs &ra,
                                   const float *fparams, const BinArgs &ba, const Outputs &out,
                                   uint32_t block, uint32_t *stage, uint32_t *cnt, uint32_t *wsum,
                                   const SharedLinear<real, DIM> &A = {}) {
  static_assert(!(GENERAL && LIN != kLinGeneral), "the shared-linear-part loop is the fast variant's");
  if constexpr (!GENERAL) flags = 0;
  const int tid = threadIdx.x;
  const uint32_t n = block * kBinBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const uint32_t plane = static_cast<uint32_t>(win.width) * static_cast<uint32_t>(win.height);

  // continued runs take the general variant (the fast one keeps its
  // registers: a fresh game from the initial point)
  real p[DIM];
  if constexpr (GENERAL)
    start_point<real, DIM>(ra, pid, n, active, out.final_points, p);
  else
    initial_point<real, DIM>(pid, ra.instance, ra.k0, ra.k1, p);
  const uint32_t blk0 = GENERAL ? ra.iter_block : 0u;
  int k = 0;
  uint32_t dropped = 0;
  int slot = 0;
  uint32_t chunk = block * ba.flushes;

  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, (t0 >> 2) + blk0, ra.instance, 0u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const uint32_t u = word_of(blk, j);
      k = select_index<SEL>(u, th, n_maps, n_search);
      if (active && out.indices)
        out.indices[static_cast<size_t>(n) * T + (t - 1)] = static_cast<uint8_t>(k);
      if constexpr (LIN != kLinGeneral)
        apply_shared_map<real, DIM, LIN>(table, A, k, p);
      else
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
        uint32_t e = kInvalid;
        if (active) {
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

  if (out.dropped && dropped)
    __hip_atomic_fetch_add(out.dropped, static_cast<unsigned long long>(dropped),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!active) return;
  if (out.final_points) {
    real *fp = static_cast<real *>(out.final_points) + static_cast<size_t>(n) * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) fp[c] = p[c];
  }
  if (out.last_index) out.last_index[n] = static_cast<uint8_t>(k);
}

// ---------------------------------------------------------------------------
// Depth images (3D camera): the stage holds (pixel | index << 24, depth bits)
// pairs; records keep the in-tile offset and the index in their first word.
// ---------------------------------------------------------------------------
__device__ inline void flush_depth_chunk(uint2 *stage, uint32_t *cnt, uint32_t *wsum, int used_slots,
                                         uint32_t chunk, const BinArgs &ba) {
  __syncthreads();
  const int tid = threadIdx.x;
  const uint32_t total = block_exclusive_scan<kDBlock>(cnt, ba.n_tiles, wsum);
  const uint32_t base = chunk * kDCap;
  uint16_t *row = ba.chunk_start + static_cast<size_t>(chunk) * (ba.n_tiles + 1);
  for (uint32_t t = tid; t <= ba.n_tiles; t += kDBlock)
    row[t] = static_cast<uint16_t>(t < ba.n_tiles ? cnt[t] : total);
  uint2 e[kDSlots];
#pragma unroll
  for (int i = 0; i < kDSlots; ++i)
    e[i] = i < used_slots ? stage[i * kDBlock + tid] : make_uint2(kInvalid, 0u);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kDSlots; ++i) {
    if (e[i].x != kInvalid) {
      const uint32_t pix = e[i].x & 0xFFFFFFu;
      stage[atomicAdd(&cnt[pix >> kDTileBits], 1u)] = e[i];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < total; i += kDBlock) {
    const uint2 v = stage[i];
    const uint32_t off = v.x & (kDTileElems - 1);
    const uint32_t k = v.x >> 24;
    ba.drecords[static_cast<size_t>(base) + i] = make_uint2(off | (k << kDTileBits), v.y);
  }
  for (uint32_t t = tid; t < ba.n_tiles; t += kDBlock) cnt[t] = 0u;
  __syncthreads();
}

// One block of kDBlock points of a 3D run with the twist/camera transform
// and the binned depth splat (same arithmetic as the direct depth path).
template <typename real, int SEL, int LIN = kLinGeneral>
__device__ void chaos_depth_block(const real *table, const uint32_t *th, int n_maps, int n_search,
                                  const Window &win, const RunArgs &ra,
                                  const real *fparams, float near_plane, const BinArgs &ba,
                                  const Outputs &out, uint32_t block, uint2 *stage, uint32_t *cnt,
                                  uint32_t *wsum, const SharedLinear<real, 3> &A = {}) {
  const int tid = threadIdx.x;
  const uint32_t n = block * kDBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  real p[3];
  start_point<real, 3>(ra, pid, n, active, out.final_points, p);
  int k = 0;
  uint32_t dropped = 0;
  int slot = 0;
  uint32_t chunk = block * ba.flushes;
  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, (t0 >> 2) + ra.iter_block, ra.instance, 0u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      k = select_index<SEL>(word_of(blk, j), th, n_maps, n_search);
      if (active && out.indices)
        out.indices[static_cast<size_t>(n) * T + (t - 1)] = static_cast<uint8_t>(k);
      if constexpr (LIN != kLinGeneral)
        apply_shared_map<real, 3, LIN>(table, A, k, p);
      else
        apply_map<real, 3>(table, k, p);
      if (t > B) {
        uint2 e = make_uint2(kInvalid, 0u);
        if (active) {
          real q[2];
          real depth = static_cast<real>(0);
          final_transform<real, kFinalTwistCamera, 3>(fparams, p, q, &depth);
          int ix;
          int pix = bin_pixel<real>(q, win, &ix);
          if (!(depth > static_cast<real>(near_plane))) pix = -1;
          if (pix >= 0)
            e = make_uint2(static_cast<uint32_t>(pix) | (static_cast<uint32_t>(k) << 24),
                           __float_as_uint(static_cast<float>(depth)));
          else
            ++dropped;
        }
        stage[slot * kDBlock + tid] = e;
        if (e.x != kInvalid) atomicAdd(&cnt[(e.x & 0xFFFFFFu) >> kDTileBits], 1u);
        if (++slot == kDSlots) {
          flush_depth_chunk(stage, cnt, wsum, slot, chunk, ba);
          slot = 0;
          ++chunk;
        }
      }
    }
  }
  if (slot > 0) flush_depth_chunk(stage, cnt, wsum, slot, chunk, ba);
  if (!active) return;
  if (out.final_points) {
    real *fp = static_cast<real *>(out.final_points) + static_cast<size_t>(n) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) fp[c] = p[c];
  }
  if (out.last_index) out.last_index[n] = static_cast<uint8_t>(k);
  if (out.dropped && dropped)
    __hip_atomic_fetch_add(out.dropped, static_cast<unsigned long long>(dropped),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Depth tile t: LDS minimum of the keys (depth bits << 32 | index) and LDS
// counts of every chunk's records of the tile, then merged into the image
// (min) and the density (sum) by the one workgroup that owns the tile.  Runs
// are walked by groups of 2^log2g lanes, each lane loading two records per
// 16-byte load from the even record at or below the run start (records
// outside [start, end) are skipped; a chunk holds an even number of records,
// so no load leaves it), kDRunsInFlight runs per group per round, kDPasses
// loads per lane and run.  The kernel waits on memory: while a round's
// records are counted, the records of the next kDAhead rounds are in flight
// and the run bounds of the round after them are loading.  Every thread
// calls it; keys and counts are kDTileElems each.
constexpr int kDRunsInFlight = 1;
constexpr int kDAhead = 1;
static_assert(kDCap % 2 == 0, "depth chunks hold whole 16-byte record pairs");

__device__ __forceinline__ void depth_record(unsigned long long *keys, uint32_t *counts,
                                             uint32_t x, uint32_t y) {
  const uint32_t off = x & (kDTileElems - 1);
  atomicMin(&keys[off], (static_cast<unsigned long long>(y) << 32) | (x >> kDTileBits));
  atomicAdd(&counts[off], 1u);
}

__device__ __forceinline__ void depth_pair(unsigned long long *keys, uint32_t *counts, uint4 v,
                                           uint32_t at, uint32_t s, uint32_t e) {
  if (at >= s && at < e) depth_record(keys, counts, v.x, v.y);
  if (at + 1u >= s && at + 1u < e) depth_record(keys, counts, v.z, v.w);
}

// Bounds [s, e) (record indices of the launch) of kDRunsInFlight runs of
// the tile: those of chunks c0, c0 + stride, ...; empty past the last chunk.
// Record indices of a launch stay below 2^31 (the launch budget).
__device__ __forceinline__ void depth_run_bounds(const uint16_t *__restrict__ row0,
                                                 const uint16_t *__restrict__ row1, uint32_t c0,
                                                 uint32_t stride, uint32_t n_chunks,
                                                 uint32_t s[kDRunsInFlight],
                                                 uint32_t e[kDRunsInFlight]) {
#pragma unroll
  for (int u = 0; u < kDRunsInFlight; ++u) {
    const uint32_t c = c0 + u * stride;
    const uint32_t base = c * kDCap;
    s[u] = c < n_chunks ? base + row0[c] : 0u;
    e[u] = c < n_chunks ? base + row1[c] : 0u;
  }
}

__device__ inline void depth_tile_accumulate(const uint2 *__restrict__ rec,
                                             const uint16_t *__restrict__ tile_start,
                                             uint32_t n_chunks, uint32_t elems,
                                             unsigned long long *__restrict__ img,
                                             uint32_t *__restrict__ density, uint32_t t,
                                             uint32_t log2g, unsigned long long *keys,
                                             uint32_t *counts) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < kDTileElems; i += kDAccBlock) {
    keys[i] = ~0ull;
    counts[i] = 0u;
  }
  __syncthreads();
  const uint16_t *row0 = tile_start + static_cast<size_t>(t) * n_chunks;
  const uint16_t *row1 = row0 + n_chunks;
  const uint32_t g = 1u << log2g, lane = tid & (g - 1u);
  const uint32_t groups = kDAccBlock >> log2g;
  const uint32_t round = groups * kDRunsInFlight;
  // ring of kDAhead + 1 rounds: bounds of rounds i .. i + kDAhead, records
  // of rounds i .. i + kDAhead - 1 issued before the loop turn of round i
  constexpr int D = kDAhead;
  constexpr int P = kDPasses;
  uint32_t s[D + 1][kDRunsInFlight], e[D + 1][kDRunsInFlight];
  uint4 v[D + 1][kDRunsInFlight][P];
  const uint32_t first = tid >> log2g;
#pragma unroll
  for (int r = 0; r <= D; ++r) depth_run_bounds(row0, row1, first + r * round, groups, n_chunks, s[r], e[r]);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int u = 0; u < kDRunsInFlight; ++u)
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const uint32_t i = (s[r][u] & ~1u) + 2u * (lane + q * g);
        v[r][u][q] = i < e[r][u] ? *reinterpret_cast<const uint4 *>(rec + i) : make_uint4(0u, 0u, 0u, 0u);
      }
  for (uint32_t c0 = first; c0 < n_chunks; c0 += round) {
    // round i + D: its records, and the bounds of the round after it
#pragma unroll
    for (int u = 0; u < kDRunsInFlight; ++u)
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const uint32_t i = (s[D][u] & ~1u) + 2u * (lane + q * g);
        v[D][u][q] = i < e[D][u] ? *reinterpret_cast<const uint4 *>(rec + i) : make_uint4(0u, 0u, 0u, 0u);
      }
    uint32_t sn[kDRunsInFlight], en[kDRunsInFlight];
    depth_run_bounds(row0, row1, c0 + (D + 1) * round, groups, n_chunks, sn, en);
    // round i: count its records (a run longer than the prefetched P * 2g
    // records continues with loads of its own)
#pragma unroll
    for (int u = 0; u < kDRunsInFlight; ++u) {
      const uint32_t i = (s[0][u] & ~1u) + 2u * lane;
#pragma unroll
      for (int q = 0; q < P; ++q)
        depth_pair(keys, counts, v[0][u][q], i + 2u * q * g, s[0][u], e[0][u]);
      for (uint32_t j = i + 2u * P * g; j < e[0][u]; j += 2u * g)
        depth_pair(keys, counts, *reinterpret_cast<const uint4 *>(rec + j), j, s[0][u], e[0][u]);
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int u = 0; u < kDRunsInFlight; ++u) {
#pragma unroll
        for (int q = 0; q < P; ++q) v[r][u][q] = v[r + 1][u][q];
        s[r][u] = s[r + 1][u];
        e[r][u] = e[r + 1][u];
      }
#pragma unroll
    for (int u = 0; u < kDRunsInFlight; ++u) {
      s[D][u] = sn[u];
      e[D][u] = en[u];
    }
  }
  __syncthreads();
  const uint32_t base = t * kDTileElems;
  const uint32_t len = min(kDTileElems, elems - base);
  for (uint32_t i = tid; i < len; i += kDAccBlock) {
    const uint32_t c = counts[i];
    if (c) {
      const unsigned long long k = keys[i];
      if (k < img[base + i]) img[base + i] = k;
      density[base + i] += c;
    }
  }
  __syncthreads();
}

// Part [c_lo, c_hi) of the chunks of image tile t: an LDS histogram of the
// tile's records in those chunks, added into the image -- with a plain
// read-modify-write when the part is every chunk (the workgroup then owns
// the tile), with device atomics when several parts share the tile.  Runs
// are walked by groups of 2^log2g lanes (one run per group, 8 records per
// lane per 16-byte load from the 8-record boundary below the run start;
// records outside [start, end) are skipped; a chunk holds a multiple of 8
// records, so no load leaves it): the group size follows the mean run
// length, so short runs keep many runs in flight and long runs are read
// with coalesced loads.  Every thread of the workgroup calls it; `tile` is
// kTileElems words of LDS.
constexpr int kRunsInFlight = 4;
static_assert(kChunkCap % 8 == 0, "chunks hold whole 16-byte record groups");

__device__ inline void count_records(uint32_t *tile, uint4 v, uint32_t at, uint32_t s,
                                     uint32_t e) {
  const uint32_t r8[8] = {v.x & 0xFFFFu, v.x >> 16, v.y & 0xFFFFu, v.y >> 16,
                          v.z & 0xFFFFu, v.z >> 16, v.w & 0xFFFFu, v.w >> 16};
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t idx = at + m;
    if (idx >= s && idx < e) atomicAdd(&tile[r8[m]], 1u);
  }
}

__device__ inline void tile_accumulate(const uint16_t *__restrict__ rec,
                                       const uint16_t *__restrict__ tile_start, uint32_t n_chunks,
                                       uint32_t c_lo, uint32_t c_hi, uint32_t elems,
                                       uint32_t *__restrict__ img, uint32_t t, uint32_t log2g,
                                       uint32_t *tile) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < kTileElems; i += kAccBlock) tile[i] = 0u;
  __syncthreads();
  const uint16_t *row0 = tile_start + static_cast<size_t>(t) * n_chunks;
  const uint16_t *row1 = row0 + n_chunks;
  const uint32_t g = 1u << log2g, lane = tid & (g - 1u);
  const uint32_t groups = kAccBlock >> log2g;
  // kRunsInFlight runs per group at a time: their bounds, then the first
  // 8g records of each, then the counts, so several loads per lane overlap
  for (uint32_t c0 = c_lo + (tid >> log2g); c0 < c_hi; c0 += groups * kRunsInFlight) {
    uint32_t s[kRunsInFlight], e[kRunsInFlight];
#pragma unroll
    for (int u = 0; u < kRunsInFlight; ++u) {
      const uint32_t c = c0 + u * groups;
      s[u] = c < c_hi ? static_cast<uint32_t>(row0[c]) : 0u;
      e[u] = c < c_hi ? static_cast<uint32_t>(row1[c]) : 0u;
    }
    // chunk bases (chunk indices and kChunkCap fit 24 bits: full-rate multiply)
#pragma unroll
    for (int u = 0; u < kRunsInFlight; ++u) {
      const uint32_t base = __umul24(c0 + u * groups, kChunkCap);
      s[u] += base;
      e[u] += base;
    }
    constexpr int P = kPasses;
    uint4 v[kRunsInFlight][P];
#pragma unroll
    for (int u = 0; u < kRunsInFlight; ++u)
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const uint32_t i = (s[u] & ~7u) + 8u * (lane + q * g);
        v[u][q] = i < e[u] ? *reinterpret_cast<const uint4 *>(rec + i) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
    for (int u = 0; u < kRunsInFlight; ++u) {
      const uint32_t i = (s[u] & ~7u) + 8u * lane;
#pragma unroll
      for (int q = 0; q < P; ++q) count_records(tile, v[u][q], i + 8u * q * g, s[u], e[u]);
      for (uint32_t j = i + 8u * P * g; j < e[u]; j += 8u * g)
        count_records(tile, *reinterpret_cast<const uint4 *>(rec + j), j, s[u], e[u]);
    }
  }
  __syncthreads();
  const uint32_t base = t * kTileElems;
  const uint32_t len = min(kTileElems, elems - base);
  const bool whole = c_lo == 0 && c_hi == n_chunks;
  for (uint32_t i = tid; i < len; i += kAccBlock) {
    const uint32_t v = tile[i];
    if (!v) continue;
    if (whole)
      img[base + i] += v;
    else
      __hip_atomic_fetch_add(img + base + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// [rows][cols] -> [cols][rows] through 64x64 LDS tiles (one workgroup of
// 256 threads per tile).  With `sums`, also the sum (mod 2^32) of each
// column over the tile's 64 rows, at sums[col * n_rb + by] (n_rb = row
// blocks): for a run-start table, tile t's record total over the chunks of
// row block by is sums[(t+1) n_rb + by] - sums[t n_rb + by].
template <typename T>
__device__ inline void transpose_tile(const T *__restrict__ in, T *__restrict__ out, uint32_t rows,
                                      uint32_t cols, uint32_t bx, uint32_t by, uint32_t (*buf)[65],
                                      uint32_t *__restrict__ sums = nullptr, uint32_t n_rb = 0) {
  const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (uint32_t r = ty; r < 64; r += 4) {
    const uint32_t gr = by * 64 + r, gc = bx * 64 + tx;
    buf[r][tx] = (gr < rows && gc < cols) ? in[static_cast<size_t>(gr) * cols + gc] : 0u;
  }
  __syncthreads();
  for (uint32_t r = ty; r < 64; r += 4) {
    const uint32_t gc = bx * 64 + r, gr = by * 64 + tx;
    if (gc < cols && gr < rows) out[static_cast<size_t>(gc) * rows + gr] = static_cast<T>(buf[tx][r]);
  }
  if (sums && ty == 0) {
    uint32_t acc = 0;  // rows past the end were loaded as zero
    for (int r = 0; r < 64; ++r) acc += buf[r][tx];
    const uint32_t gc = bx * 64 + tx;
    if (gc < cols) sums[static_cast<size_t>(gc) * n_rb + by] = acc;
  }
  __syncthreads();
}

}  // namespace cfs
