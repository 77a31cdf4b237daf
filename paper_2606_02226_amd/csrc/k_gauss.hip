// k_gauss.hip -- differentiable form of the chaos game (Section 4 of the
// paper: the distribution of a primitive could be generated automatically with
// autodiff-like tools).
//
// Forward: the chaos game of a 2D affine system in FP32 splats every iterate
// with a separable shifted-truncated Gaussian (continuous in the point, so the
// density is a continuous function of the map parameters).  Like the integer
// splat, the taps are not applied with device atomics: each splat becomes one
// (x, y) record, records are sorted in LDS by the 32x32-pixel tile that holds
// their footprint's first tap, and per-tile workgroups sum the taps of their
// tile's records as integers into an LDS tile with a margin of TAPS - 1
// pixels on every side (a footprint of at most 16 taps reaches at most that
// far past its tile), then add it to the density.  Checkpoints of the
// positions every c iterations are written for the backward pass.
//
// Backward: the records are emitted again, each with its index per (step,
// point); per-tile workgroups compute every splat's gradient s_t from an LDS
// copy of dL/dD; then per point each checkpoint segment is recomputed into
// registers and swept in reverse with the adjoint
//   lam_t = s_t + A_{k_{t+1}}^T lam_{t+1},  dA_{k_t} += lam_t p_{t-1}^T,
//   db_{k_t} += lam_t.
// Gradients stay in registers per lane and are reduced in a fixed order (no
// floating-point atomics).
#include "cfs_device.hpp"
#include "cfs_host.hpp"

namespace cfs {

constexpr uint32_t kGInvalid = 0xFFFFFFFFu;
constexpr int kGWaves = kGBlock / 64;

__device__ __forceinline__ bool rec_valid(float2 r) { return __float_as_uint(r.x) != kGInvalid; }

// First tap index of a point at pixel coordinate x: taps i satisfy
// |i + 0.5 - x| < R, i.e. i > x - R - 0.5.
__device__ __forceinline__ int first_tap(float x, float R) {
  return static_cast<int>(floorf(x - R - 0.5f)) + 1;
}

__device__ __forceinline__ uint32_t gauss_tile_of(float2 r, const GaussParams &gp) {
  const int i0 = max(first_tap(r.x, gp.R), 0);
  const int j0 = max(first_tap(r.y, gp.R), 0);
  return static_cast<uint32_t>((j0 >> kGTileLog) * gp.tiles_x + (i0 >> kGTileLog));
}

constexpr int kGScanPer = (kGMaxTiles + kGBlock - 1) / kGBlock;

__device__ uint32_t gblock_exclusive_scan(uint32_t *a, uint32_t n, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t i0 = static_cast<uint32_t>(tid) * kGScanPer;
  uint32_t v[kGScanPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kGScanPer; ++q) {
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
    const uint32_t x = lane < kGWaves ? wsum[lane] : 0u;
    uint32_t xi = x;
#pragma unroll
    for (int d = 1; d < kGWaves; d <<= 1) {
      const uint32_t y = __shfl_up(xi, d, 64);
      if (lane >= d) xi += y;
    }
    if (lane < kGWaves) wsum[lane] = xi - x;
    if (lane == kGWaves - 1) wsum[kGWaves] = xi;
  }
  __syncthreads();
  uint32_t run = wsum[w] + incl - s;
#pragma unroll
  for (int q = 0; q < kGScanPer; ++q) {
    if (i0 + q < n) a[i0 + q] = run;
    run += v[q];
  }
  const uint32_t total = wsum[kGWaves];
  __syncthreads();
  return total;
}

// POS: also write, for every splat of the flush (points of the launch slice
// only), the index of its record, or kGInvalid for a splat off the image, at
// pos[iteration - B - 1][point]: the adjoint reads each splat's gradient
// there after the per-tile kernel has written it in record order.
template <bool POS>
__device__ void gauss_flush(float2 *stage, uint32_t *cnt, uint32_t *wsum, int used, uint32_t chunk,
                            uint32_t points, const GaussParams &gp, const GaussBin &gb) {
  __syncthreads();
  const int tid = threadIdx.x;
  float2 e[kGSlots];
  uint32_t tl[kGSlots], r[kGSlots];
#pragma unroll
  for (int i = 0; i < kGSlots; ++i) {
    e[i] = i < used ? stage[i * kGBlock + tid] : make_float2(__uint_as_float(kGInvalid), 0.f);
    tl[i] = rec_valid(e[i]) ? gauss_tile_of(e[i], gp) : kGInvalid;
    r[i] = tl[i] != kGInvalid ? atomicAdd(&cnt[tl[i]], 1u) : 0u;
  }
  __syncthreads();  // every count complete before the scan reads them
  const uint32_t total = gblock_exclusive_scan(cnt, gb.n_tiles, wsum);
  const uint32_t base = chunk * kGCap;
  uint32_t *row = gb.chunk_start + static_cast<size_t>(chunk) * (gb.n_tiles + 1);
  for (uint32_t t = tid; t <= gb.n_tiles; t += kGBlock) row[t] = base + (t < gb.n_tiles ? cnt[t] : total);
  if constexpr (POS) {
    const uint32_t f = chunk % gb.flushes;
    const uint32_t n = (chunk / gb.flushes) * kGBlock + tid;
    if (n < points) {
#pragma unroll
      for (int i = 0; i < kGSlots; ++i)
        if (i < used)
          gb.pos[static_cast<size_t>(f * kGSlots + i) * points + n] =
              tl[i] != kGInvalid ? base + cnt[tl[i]] + r[i] : kGInvalid;
    }
  }
#pragma unroll
  for (int i = 0; i < kGSlots; ++i)
    if (tl[i] != kGInvalid) stage[cnt[tl[i]] + r[i]] = e[i];
  __syncthreads();
  for (uint32_t i = tid; i < total; i += kGBlock) gb.records[static_cast<size_t>(base) + i] = stage[i];
  __syncthreads();
  for (uint32_t t = tid; t < gb.n_tiles; t += kGBlock) cnt[t] = 0u;
  __syncthreads();
}

template <bool EQUAL, bool POS>
__global__ __launch_bounds__(kGBlock) void k_splat_emit(MapTable<2> mt, RunArgs ra, GaussParams gp,
                                                        GaussBin gb, GaussCkpt ck,
                                                        unsigned long long *dropped_out) {
  __shared__ float table[kMaxMaps * 8];
  __shared__ uint32_t th[kThWords];
  __shared__ float2 stage[kGCap];
  __shared__ uint32_t cnt[kGMaxTiles];
  __shared__ uint32_t wsum[kGWaves + 1];
  const int tid = threadIdx.x;
  load_table<float, 2>(mt, table, th);
  for (uint32_t t = tid; t < gb.n_tiles; t += kGBlock) cnt[t] = 0u;
  __syncthreads();

  const uint32_t n = blockIdx.x * kGBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  float p[2];
  initial_point<float, 2>(pid, ra.instance, ra.k0, ra.k1, p);
  if (active && ck.ckpt) reinterpret_cast<float2 *>(ck.ckpt)[n] = make_float2(p[0], p[1]);
  uint32_t dropped = 0;
  int slot = 0;
  uint32_t chunk = blockIdx.x * gb.flushes;
  const float lim = gp.R + 16.0f;

  for (uint32_t t0 = 0; t0 < T; t0 += 4) {
    const Block4 blk = philox10(pid, t0 >> 2, ra.instance, 0u, ra.k0, ra.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + j + 1;
      if (t > T) break;
      const uint32_t u = word_of(blk, j);
      int k;
      if constexpr (EQUAL)
        k = select_equal(u, static_cast<uint32_t>(mt.n_maps));
      else
        k = select_table(u, th);
      apply_map<float, 2>(table, k, p);
      if (active && ck.ckpt && t < T && t % ck.every == 0)
        reinterpret_cast<float2 *>(ck.ckpt)[static_cast<size_t>(t / ck.every) * ck.stride + n] =
            make_float2(p[0], p[1]);
      if (t > B) {
        float2 rec = make_float2(__uint_as_float(kGInvalid), 0.f);
        if (active) {
          const float x = (p[0] - gp.lo[0]) * gp.scale[0];
          const float y = (p[1] - gp.lo[1]) * gp.scale[1];
          if (x > -lim && x < gp.width + lim && y > -lim && y < gp.height + lim) {
            const int i0 = first_tap(x, gp.R), j0 = first_tap(y, gp.R);
            if (i0 + gp.taps - 1 >= 0 && i0 <= gp.width - 1 && j0 + gp.taps - 1 >= 0 &&
                j0 <= gp.height - 1)
              rec = make_float2(x, y);
          }
          if (!rec_valid(rec)) ++dropped;
        }
        stage[slot * kGBlock + tid] = rec;
        if (++slot == kGSlots) {
          gauss_flush<POS>(stage, cnt, wsum, slot, chunk, ra.n_points, gp, gb);
          slot = 0;
          ++chunk;
        }
      }
    }
  }
  if (slot > 0) gauss_flush<POS>(stage, cnt, wsum, slot, chunk, ra.n_points, gp, gb);
  if (active && dropped_out && dropped)
    __hip_atomic_fetch_add(dropped_out, static_cast<unsigned long long>(dropped), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

constexpr float kLog2E = 1.44269504088896341f;

// Offsets d_a = i0 + a + 0.5 - x of the TAPS candidate taps from i0 (as a - u
// with u = x - i0 - 0.5, one subtraction per tap), and exp(-d_a^2 / 2 s^2)
// as exp2(d_a^2 k) with k = -log2(e) / 2 s^2.
template <int TAPS>
__device__ __forceinline__ void tap_gauss(float x, int i0, const GaussParams &gp, float d[TAPS],
                                          float e[TAPS]) {
  const float u = x - (static_cast<float>(i0) + 0.5f);
  const float k = -gp.inv2s2 * kLog2E;
#pragma unroll
  for (int a = 0; a < TAPS; ++a) {
    d[a] = static_cast<float>(a) - u;
    e[a] = __builtin_amdgcn_exp2f(d[a] * d[a] * k);
  }
}

// Tap weights g(i + 0.5 - x) for the TAPS candidate taps from i0; taps at
// distance R or more get weight 0.  Candidates off the image keep their
// weight: the callers drop them (LDS cells that are never flushed, or a zero
// upstream gradient).
template <int TAPS>
__device__ __forceinline__ void tap_weights(float x, int i0, const GaussParams &gp, float g[TAPS]) {
  float d[TAPS], e[TAPS];
  tap_gauss<TAPS>(x, i0, gp, d, e);
#pragma unroll
  for (int a = 0; a < TAPS; ++a) g[a] = fabsf(d[a]) < gp.R ? e[a] - gp.cutoff : 0.0f;
}

// The part of its tile that workgroup b of a per-tile launch takes.  Each
// tile has p_max consecutive workgroups (consecutive blocks go to different
// XCDs, so the parts of a dense tile spread over the chip); the tile uses
// ceil(total / per_part) of them, at most p_max, each with an equal share of
// the chunks.  Returns false (the same in every lane) for a workgroup the
// tile does not use.  `sums` holds the transpose's column sums of 64-chunk
// blocks.
struct TilePart {
  uint32_t t, c_lo, c_hi;
};
__device__ inline bool gauss_tile_part(const uint32_t *__restrict__ sums, uint32_t n_rb,
                                       uint32_t n_chunks, uint32_t p_max, uint32_t per_part,
                                       TilePart *tp) {
  __shared__ uint32_t red[kGAccBlock / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t t = blockIdx.x / p_max, part = blockIdx.x % p_max;
  const uint32_t *lo = sums + static_cast<size_t>(t) * n_rb, *hi = lo + n_rb;
  uint32_t s = 0;
  for (uint32_t b = tid; b < n_rb; b += kGAccBlock) s += hi[b] - lo[b];
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  uint32_t total = 0;
#pragma unroll
  for (int w = 0; w < kGAccBlock / 64; ++w) total += red[w];
  const uint32_t parts = min(p_max, (total + per_part - 1) / per_part);
  if (part >= parts) return false;
  tp->t = t;
  tp->c_lo = static_cast<uint32_t>(static_cast<uint64_t>(n_chunks) * part / parts);
  tp->c_hi = static_cast<uint32_t>(static_cast<uint64_t>(n_chunks) * (part + 1) / parts);
  return true;
}

// The records of a workgroup's tile and chunk range: at most 2^32 - 1 (a
// tile's records in one launch never reach 2^32).
__device__ inline uint32_t gauss_part_records(const uint32_t *row0, const uint32_t *row1,
                                              const TilePart &tp) {
  __shared__ uint32_t red[kGAccBlock / 64];
  uint32_t n = 0;
  for (uint32_t c = tp.c_lo + threadIdx.x; c < tp.c_hi; c += kGAccBlock) n += row1[c] - row0[c];
  for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = n;
  __syncthreads();
  uint32_t total = 0;
#pragma unroll
  for (int w = 0; w < kGAccBlock / 64; ++w) total += red[w];
  return total;
}

// Calls f(i, rec[i]) once for every record i of a workgroup's tile and chunk
// range.  The runs are taken kGAccBlock at a time: their lengths are scanned
// into LDS and the batch's records dealt out evenly, lane j taking records
// j, j + kGAccBlock, ... of the batch (each found by a binary search over the
// runs' prefix sums), so no lane idles on short or uneven runs.  A lane loads
// its next record before it handles the current one.
template <typename F>
__device__ __forceinline__ void gauss_part_walk(const float2 *__restrict__ rec, const uint32_t *row0,
                                                const uint32_t *row1, const TilePart &tp, F &&f) {
  __shared__ uint32_t run_s[kGAccBlock];  // first record of each run of the batch
  __shared__ uint32_t run_p[kGAccBlock];  // records of the batch before each run
  __shared__ uint32_t wtot[kGAccBlock / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  for (uint32_t c0 = tp.c_lo; c0 < tp.c_hi; c0 += kGAccBlock) {
    const uint32_t c = c0 + tid;
    const uint32_t s = c < tp.c_hi ? row0[c] : 0u;
    const uint32_t len = c < tp.c_hi ? row1[c] - s : 0u;
    uint32_t incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= static_cast<uint32_t>(d)) incl += y;
    }
    if (lane == 63u) wtot[w] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t v = 0; v < kGAccBlock / 64; ++v) {
      const uint32_t x = wtot[v];
      before += v < w ? x : 0u;
      total += x;
    }
    run_s[tid] = s;
    run_p[tid] = before + incl - len;
    __syncthreads();
    // record k of the batch: run r is the last with run_p[r] <= k (k < total,
    // so r has records and k - run_p[r] is less than its length)
    auto locate = [&](uint32_t k) {
      uint32_t r = 0;
#pragma unroll
      for (uint32_t step = kGAccBlock / 2; step >= 1; step >>= 1)
        if (run_p[r + step] <= k) r += step;
      return run_s[r] + (k - run_p[r]);
    };
    uint32_t k = tid, i = 0;
    float2 r = make_float2(0.0f, 0.0f);
    if (k < total) {
      i = locate(k);
      r = rec[i];
    }
    while (k < total) {
      const uint32_t k2 = k + kGAccBlock;
      uint32_t i2 = 0;
      float2 r2 = make_float2(0.0f, 0.0f);
      if (k2 < total) {
        i2 = locate(k2);
        r2 = rec[i2];
      }
      f(i, r);
      k = k2;
      i = i2;
      r = r2;
    }
    __syncthreads();  // the batch's tables are read up to here
  }
}

// One workgroup per (tile, chunk range): the records of its own tile only
// (binned by their first tap, so every footprint starts at most TAPS - 1
// pixels left of or above the tile, off the image there, and ends at most
// TAPS - 1 pixels past its right and lower edges) are read once and their
// taps summed into an LDS tile with those margins.  The LDS sums are 32-bit
// integers: each tap adds round(g(dx) g(dy) 2^s) with s = clz(C) for the C
// records of the workgroup, so that C taps of weight at most 1 (each record
// adds at most one tap to a pixel) stay below 2^32: C < 2^(32 - s).  32-bit
// LDS integer atomics run at about twice the rate of 64-bit ones and far
// faster than floating-point ones, and integer sums do not depend on their
// order; a tap is held to 2^-(s+1), and s >= 21 for parts of up to 2047
// records (the usual size).
// Every tap adds, also those of weight 0, so the loop has no branches and
// its LDS addresses are one base plus constant offsets.  The tile plus its
// right and lower halo is then scaled by 2^-s / (N (T - B)) and added into
// the density with device float atomics (neighbouring tiles and the other
// chunk ranges of the tile add into the same pixels).
template <int TAPS>
__global__ __launch_bounds__(kGAccBlock) void k_splat_accumulate(const float2 *__restrict__ rec,
                                                                 const uint32_t *__restrict__ tile_start,
                                                                 const uint32_t *__restrict__ sums,
                                                                 uint32_t n_rb, uint32_t n_chunks,
                                                                 uint32_t p_max, uint32_t per_part,
                                                                 GaussParams gp,
                                                                 float *__restrict__ dens) {
  constexpr int H = kGTile + TAPS - 1;  // tile plus right and lower halo, per axis
  constexpr int M = TAPS - 1;           // margin left of and above the tile
  constexpr int HM = H + M;
  __shared__ uint32_t acc[HM * HM];
  TilePart tp;
  if (!gauss_tile_part(sums, n_rb, n_chunks, p_max, per_part, &tp)) return;
  const uint32_t tid = threadIdx.x;
  const int tx = tp.t % gp.tiles_x, ty = tp.t / gp.tiles_x;
  const int x0 = tx * kGTile, y0 = ty * kGTile;
  for (uint32_t i = tid; i < HM * HM; i += kGAccBlock) acc[i] = 0u;
  const uint32_t *row0 = tile_start + static_cast<size_t>(tp.t) * n_chunks;
  const uint32_t *row1 = row0 + n_chunks;
  const uint32_t n_rec = gauss_part_records(row0, row1, tp);  // synchronises the clear too
  const int sh = n_rec ? __clz(n_rec) : 31;
  const float scale = __uint_as_float(static_cast<uint32_t>(127 + sh) << 23);  // 2^sh
  gauss_part_walk(rec, row0, row1, tp, [&](uint32_t, float2 r) {
    const int i0 = first_tap(r.x, gp.R), j0 = first_tap(r.y, gp.R);
    // taps left of or above the tile are off the image (first taps are
    // clamped to 0 for binning) and land in the margins; taps past the
    // image's right or lower edge land in halo cells outside the image:
    // neither is flushed
    float gx[TAPS], gy[TAPS];
    tap_weights<TAPS>(r.x, i0, gp, gx);
    tap_weights<TAPS>(r.y, j0, gp, gy);
    uint32_t *base = acc + (j0 - y0 + M) * HM + (i0 - x0 + M);
#pragma unroll
    for (int b = 0; b < TAPS; ++b) {
      const float wy = gy[b] * scale;  // g <= 1 per axis
      // round to nearest: truncate the product plus 1/2 (gx wy < 2^s, so
      // the tap is at most 2^s)
#pragma unroll
      for (int a = 0; a < TAPS; ++a)
        atomicAdd(base + b * HM + a, static_cast<uint32_t>(fmaf(gx[a], wy, 0.5f)));
    }
  });
  const double unit = ldexp(static_cast<double>(gp.weight), -sh);
  for (uint32_t i = tid; i < H * H; i += kGAccBlock) {
    const int px = x0 + static_cast<int>(i % H), py = y0 + static_cast<int>(i / H);
    const uint32_t v = acc[(i / H + M) * HM + i % H + M];
    if (px < gp.width && py < gp.height && v != 0u)
      atomicAdd(dens + static_cast<size_t>(py) * gp.width + px,
                static_cast<float>(static_cast<double>(v) * unit));
  }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
// dL/dx, dL/dy (in pixels, before the chain to positions) of one splat at
// pixel coordinates (x, y): the taps' weights g and derivatives dg against
// the upstream gradient G, read through `at(row, col)` for every candidate
// tap.  `at` must accept every candidate and return 0 for those off the
// image, and taps at distance R or more get g = dg = 0, so every tap without
// a weight adds an exact zero and the sums are those over the image's taps.
template <int TAPS, typename GAt>
__device__ __forceinline__ void splat_grad_px(float x, float y, const GaussParams &gp, GAt at,
                                              float *ax_out, float *ay_out) {
  const int i0 = first_tap(x, gp.R), j0 = first_tap(y, gp.R);
  float gx[TAPS], dgx[TAPS], gy[TAPS], dgy[TAPS];
  {
    float dx[TAPS], ex[TAPS], dy[TAPS], ey[TAPS];
    tap_gauss<TAPS>(x, i0, gp, dx, ex);
    tap_gauss<TAPS>(y, j0, gp, dy, ey);
#pragma unroll
    for (int a = 0; a < TAPS; ++a) {
      const bool on = fabsf(dx[a]) < gp.R;
      gx[a] = on ? ex[a] - gp.cutoff : 0.0f;
      dgx[a] = on ? -dx[a] * gp.inv_s2 * ex[a] : 0.0f;
      const bool ony = fabsf(dy[a]) < gp.R;
      gy[a] = ony ? ey[a] - gp.cutoff : 0.0f;
      dgy[a] = ony ? -dy[a] * gp.inv_s2 * ey[a] : 0.0f;
    }
  }
  float ax = 0.0f, ay = 0.0f;
#pragma unroll
  for (int b = 0; b < TAPS; ++b) {
    float sg = 0.0f, sdg = 0.0f;
#pragma unroll
    for (int a = 0; a < TAPS; ++a) {
      const float v = at(j0 + b, i0 + a);
      sg += v * gx[a];
      sdg += v * dgx[a];
    }
    ax += gy[b] * sdg;
    ay += dgy[b] * sg;
  }
  *ax_out = ax;
  *ay_out = ay;
}

// Per record of one tile and chunk range: the gradient of the loss with
// respect to the splatted position, from an LDS copy of the tile's upstream
// gradient with the same halo and margins as the forward accumulate (the
// margin left of and above the tile holds zeros), written to
// S at the record's own index (coalesced; the adjoint finds it through the
// emit's pos map).  Workgroups, tile parts and lane groups as in the forward
// accumulate.
template <int TAPS>
__global__ __launch_bounds__(kGAccBlock) void k_splat_grad_tiles(
    const float2 *__restrict__ rec, const uint32_t *__restrict__ tile_start,
    const uint32_t *__restrict__ sums, uint32_t n_rb, uint32_t n_chunks, uint32_t p_max,
    uint32_t per_part, GaussParams gp,
    const float *__restrict__ G, float2 *__restrict__ S) {
  constexpr int H = kGTile + TAPS - 1;
  constexpr int M = TAPS - 1;
  constexpr int HM = H + M;
  __shared__ float g[HM * HM];
  TilePart tp;
  if (!gauss_tile_part(sums, n_rb, n_chunks, p_max, per_part, &tp)) return;
  const uint32_t tid = threadIdx.x;
  const int tx = tp.t % gp.tiles_x, ty = tp.t / gp.tiles_x;
  const int x0 = tx * kGTile, y0 = ty * kGTile;
  for (uint32_t i = tid; i < HM * HM; i += kGAccBlock) {
    const int ox = static_cast<int>(i % HM) - M, oy = static_cast<int>(i / HM) - M;
    const int px = x0 + ox, py = y0 + oy;
    g[i] = (ox >= 0 && oy >= 0 && px < gp.width && py < gp.height)
               ? G[static_cast<size_t>(py) * gp.width + px]
               : 0.0f;
  }
  __syncthreads();
  // every candidate tap lies in [x0 - M, x0 + H) x [y0 - M, y0 + H) (records
  // are binned by their first tap; taps left of or above the tile are off the
  // image and read the zero margin, taps past its right or lower edge read
  // the zeros loaded there)
  auto at = [&](int row, int col) { return g[(row - y0 + M) * HM + (col - x0 + M)]; };
  const float cx = -gp.scale[0] * gp.weight, cy = -gp.scale[1] * gp.weight;
  const uint32_t *row0 = tile_start + static_cast<size_t>(tp.t) * n_chunks;
  const uint32_t *row1 = row0 + n_chunks;
  gauss_part_walk(rec, row0, row1, tp, [&](uint32_t i, float2 r) {
    float ax, ay;
    splat_grad_px<TAPS>(r.x, r.y, gp, at, &ax, &ay);
    S[i] = make_float2(ax * cx, ay * cy);
  });
}

// The adjoint sweep of each point of a launch slice, with the splat
// gradients already computed per tile: splat t of point n has its gradient
// at S[pos[t - B - 1][n]] (none if pos holds kGInvalid: off the image).
// SEG bounds the checkpoint interval: a segment's positions and map indices
// stay in registers (3 (SEG + 1) of them), so the common intervals up to 8
// take a kernel with half the live registers (twice the resident waves to
// hide the gathers of S) of the one for intervals up to 16.
template <int NG, bool EQUAL, int SEG>
__global__ __launch_bounds__(kGBwdBlock) void k_splat_backward(MapTable<2> mt, RunArgs ra,
                                                               const uint32_t *__restrict__ pos,
                                                               const float2 *__restrict__ S,
                                                               GaussCkpt ck, float *partials,
                                                               uint32_t block_offset) {
  __shared__ float table[kMaxMaps * 8];
  __shared__ uint32_t th[kThWords];
  __shared__ float red[kGBwdBlock / 64][NG * 6];
  load_table<float, 2>(mt, table, th);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t n = blockIdx.x * kGBwdBlock + tid;
  const bool active = n < ra.n_points;
  const uint32_t pid = ra.point_offset + (active ? n : 0u);
  const uint32_t T = ra.n_iters, B = ra.burn_in;
  const uint32_t c = static_cast<uint32_t>(ck.every);
  float g[NG][6];
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int q = 0; q < 6; ++q) g[m][q] = 0.0f;

  if (active) {
    float lam0 = 0.0f, lam1 = 0.0f;
    int k_next = -1;
    const uint32_t n_seg = (T + c - 1) / c;
    for (int seg = static_cast<int>(n_seg) - 1; seg >= 0; --seg) {
      const uint32_t t_start = static_cast<uint32_t>(seg) * c;
      const uint32_t len = min(c, T - t_start);
      float px[SEG + 1], py[SEG + 1];
      int ks[SEG + 1];
      const float2 p0 = reinterpret_cast<const float2 *>(ck.ckpt)[static_cast<size_t>(seg) * ck.stride + n];
      px[0] = p0.x;
      py[0] = p0.y;
      ks[0] = 0;
      // the segment's splat gradients, gathered first so that their latency
      // hides under the recompute (the gathers do not depend on it)
      float2 sv[SEG + 1];
#pragma unroll
      for (int m = 1; m <= SEG; ++m) {
        const uint32_t t = t_start + m;
        uint32_t q = kGInvalid;
        if (static_cast<uint32_t>(m) <= len && t > B)
          q = pos[static_cast<size_t>(t - B - 1) * ra.n_points + n];
        sv[m] = q != kGInvalid ? S[q] : make_float2(0.0f, 0.0f);
      }
      // recompute the segment exactly as the forward pass did
      Block4 blk{0u, 0u, 0u, 0u};
      float p[2] = {p0.x, p0.y};
#pragma unroll
      for (int m = 1; m <= SEG; ++m) {
        if (static_cast<uint32_t>(m) > len) break;
        const uint32_t t = t_start + m;
        if (m == 1 || ((t - 1) & 3u) == 0u)
          blk = philox10(pid, (t - 1) >> 2, ra.instance, 0u, ra.k0, ra.k1);
        const uint32_t u = word_of(blk, static_cast<int>((t - 1) & 3u));
        int k;
        if constexpr (EQUAL)
          k = select_equal(u, static_cast<uint32_t>(mt.n_maps));
        else
          k = select_table(u, th);
        apply_map<float, 2>(table, k, p);
        px[m] = p[0];
        py[m] = p[1];
        ks[m] = k;
      }
      // reverse sweep
#pragma unroll
      for (int m = SEG; m >= 1; --m) {
        if (static_cast<uint32_t>(m) > len) continue;
        const float s0 = sv[m].x, s1 = sv[m].y;
        float c0 = 0.0f, c1 = 0.0f;
        if (k_next >= 0) {
          const float *A = table + k_next * 8;  // a00 a01 a10 a11: A^T lam
          c0 = A[0] * lam0 + A[2] * lam1;
          c1 = A[1] * lam0 + A[3] * lam1;
        }
        lam0 = s0 + c0;
        lam1 = s1 + c1;
        const int k = ks[m];
        const float q0 = px[m - 1], q1 = py[m - 1];
#pragma unroll
        for (int mm = 0; mm < NG; ++mm) {
          const float sel = (k == mm) ? 1.0f : 0.0f;
          const float l0 = sel * lam0, l1 = sel * lam1;
          g[mm][0] += l0 * q0;
          g[mm][1] += l0 * q1;
          g[mm][2] += l1 * q0;
          g[mm][3] += l1 * q1;
          g[mm][4] += l0;
          g[mm][5] += l1;
        }
        k_next = k;
      }
    }
  }
  // fixed-order reduction: butterfly within the wave, then waves in order
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      float v = g[m][q];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
      if (lane == 0) red[w][m * 6 + q] = v;
    }
  __syncthreads();
  if (tid < NG * 6) {
    float s = 0.0f;
    for (int ww = 0; ww < kGBwdBlock / 64; ++ww) s += red[ww][tid];
    partials[static_cast<size_t>(block_offset + blockIdx.x) * (NG * 6) + tid] = s;
  }
}

// grad[i] = the FP64 sum over workgroups b of partials[b][i], one workgroup
// per entry i: thread j sums the workgroups b = j (mod 256) in order, then a
// fixed tree adds the 256 sums, so the result depends only on the inputs.
constexpr int kReduceBlock = 256;

__global__ __launch_bounds__(kReduceBlock) void k_grad_reduce(const float *partials, uint32_t blocks,
                                                              int ng6, float *grad) {
  __shared__ double lds[kReduceBlock];
  const int i = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (uint32_t b = tid; b < blocks; b += kReduceBlock)
    s += static_cast<double>(partials[static_cast<size_t>(b) * ng6 + i]);
  lds[tid] = s;
  __syncthreads();
  for (int w = kReduceBlock / 2; w > 0; w >>= 1) {
    if (tid < w) lds[tid] += lds[tid + w];
    __syncthreads();
  }
  if (tid == 0) grad[i] = static_cast<float>(lds[0]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
GaussPlan gauss_plan(uint32_t points, uint32_t n_iters, uint32_t burn_in, int width, int height) {
  GaussPlan gp{};
  gp.blocks = (points + kGBlock - 1) / kGBlock;
  gp.flushes = (n_iters - burn_in + kGSlots - 1) / kGSlots;
  gp.n_chunks = gp.blocks * gp.flushes;
  gp.tiles_x = (width + kGTile - 1) / kGTile;
  gp.tiles_y = (height + kGTile - 1) / kGTile;
  gp.n_tiles = static_cast<uint32_t>(gp.tiles_x) * gp.tiles_y;
  gp.n_rb = (gp.n_chunks + 63) / 64;
  gp.records_bytes = static_cast<size_t>(gp.n_chunks) * kGCap * sizeof(float2);
  gp.table_bytes = static_cast<size_t>(gp.n_tiles + 1) * gp.n_chunks * sizeof(uint32_t);
  gp.sums_bytes = static_cast<size_t>(gp.n_tiles + 1) * gp.n_rb * sizeof(uint32_t);
  return gp;
}

// Per-tile kernels' launch shape: p_max workgroups per tile (at most
// kGMaxParts, fewer on images of many tiles so that the grid stays near
// 32768 workgroups, most of which end at once), and a workgroup per
// per_part records, per_part being the launch's splats (an upper bound on
// its records) over kGPartTarget, so that dense tiles take many small
// workgroups whatever the spread of the work over the tiles.
static void gauss_tile_shape(const GaussJob &j, uint32_t *p_max_out, uint32_t *per_part_out) {
  const uint32_t p_max = std::min<uint32_t>(kGMaxParts, std::max<uint32_t>(8u, 32768u / j.gb.n_tiles));
  const uint64_t splats = static_cast<uint64_t>(j.ra.n_points) * (j.ra.n_iters - j.ra.burn_in);
  const uint64_t per_part = (splats + kGPartTarget - 1) / kGPartTarget;
  *p_max_out = p_max;
  *per_part_out = static_cast<uint32_t>(std::max<uint64_t>(per_part, 1));
}

template <bool POS>
static hipError_t launch_emit(const GaussJob &j, const GaussCkpt &ck, unsigned long long *dropped,
                              hipStream_t s) {
  const uint32_t blocks = (j.ra.n_points + kGBlock - 1) / kGBlock;
  if (j.equal)
    hipLaunchKernelGGL((k_splat_emit<true, POS>), dim3(blocks), dim3(kGBlock), 0, s, j.mt, j.ra, j.gp,
                       j.gb, ck, dropped);
  else
    hipLaunchKernelGGL((k_splat_emit<false, POS>), dim3(blocks), dim3(kGBlock), 0, s, j.mt, j.ra, j.gp,
                       j.gb, ck, dropped);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_transpose(j.gb.chunk_start, j.gb.tile_start, j.gb.n_chunks, j.gb.n_tiles + 1, s,
                          j.gb.tile_sums);
}

hipError_t launch_splat_forward(const GaussJob &j, hipStream_t s) {
  if (j.ra.n_points == 0) return hipSuccess;
  if (j.gb.n_chunks == 0) {
    // no step is splatted (burn_in == n_iters): the emit kernel still walks
    // the trajectory for its checkpoints; it stages nothing and never
    // flushes, and the transpose of a table without rows is a no-op
    return j.ck.ckpt ? launch_emit<false>(j, j.ck, j.dropped, s) : hipSuccess;
  }
  hipError_t e = launch_emit<false>(j, j.ck, j.dropped, s);
  if (e != hipSuccess) return e;
  uint32_t p_max, per_part;
  gauss_tile_shape(j, &p_max, &per_part);
  const dim3 grid(j.gb.n_tiles * p_max);
  if (j.gp.taps <= 6)
    hipLaunchKernelGGL(k_splat_accumulate<6>, grid, dim3(kGAccBlock), 0, s, j.gb.records,
                       j.gb.tile_start, j.gb.tile_sums, j.gb.n_rb, j.gb.n_chunks, p_max, per_part,
                       j.gp, j.dens);
  else
    hipLaunchKernelGGL(k_splat_accumulate<16>, grid, dim3(kGAccBlock), 0, s, j.gb.records,
                       j.gb.tile_start, j.gb.tile_sums, j.gb.n_rb, j.gb.n_chunks, p_max, per_part,
                       j.gp, j.dens);
  return hipGetLastError();
}

template <int NG, int SEG>
static void launch_sweep(const GaussJob &j, uint32_t block_offset, hipStream_t s) {
  const uint32_t blocks = (j.ra.n_points + kGBwdBlock - 1) / kGBwdBlock;
  if (j.equal)
    hipLaunchKernelGGL((k_splat_backward<NG, true, SEG>), dim3(blocks), dim3(kGBwdBlock), 0, s, j.mt,
                       j.ra, j.gb.pos, j.S, j.ck, j.partials, block_offset);
  else
    hipLaunchKernelGGL((k_splat_backward<NG, false, SEG>), dim3(blocks), dim3(kGBwdBlock), 0, s, j.mt,
                       j.ra, j.gb.pos, j.S, j.ck, j.partials, block_offset);
}

template <int NG>
static void launch_sweep(const GaussJob &j, uint32_t block_offset, hipStream_t s) {
  if (j.ck.every <= kShortSeg)
    launch_sweep<NG, kShortSeg>(j, block_offset, s);
  else
    launch_sweep<NG, kMaxSeg>(j, block_offset, s);
}

hipError_t launch_splat_backward_slice(const GaussJob &j, uint32_t block_offset, hipStream_t s) {
  if (j.ra.n_points == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (j.gb.n_chunks) {
    // the slice's records again with the record index of every splat, then
    // the splat gradients per tile, in record order
    const GaussCkpt none{nullptr, 1, 0};
    e = launch_emit<true>(j, none, nullptr, s);
    if (e != hipSuccess) return e;
    uint32_t p_max, per_part;
    gauss_tile_shape(j, &p_max, &per_part);
    const dim3 grid(j.gb.n_tiles * p_max);
    if (j.gp.taps <= 6)
      hipLaunchKernelGGL(k_splat_grad_tiles<6>, grid, dim3(kGAccBlock), 0, s, j.gb.records,
                         j.gb.tile_start, j.gb.tile_sums, j.gb.n_rb, j.gb.n_chunks, p_max, per_part,
                         j.gp, j.dLdD, j.S);
    else
      hipLaunchKernelGGL(k_splat_grad_tiles<16>, grid, dim3(kGAccBlock), 0, s, j.gb.records,
                         j.gb.tile_start, j.gb.tile_sums, j.gb.n_rb, j.gb.n_chunks, p_max, per_part,
                         j.gp, j.dLdD, j.S);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (j.mt.n_maps <= 4)
    launch_sweep<4>(j, block_offset, s);
  else
    launch_sweep<8>(j, block_offset, s);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const GaussJob &j, uint32_t blocks, hipStream_t s) {
  const int ng = j.mt.n_maps <= 4 ? 4 : 8;
  hipLaunchKernelGGL(k_grad_reduce, dim3(j.mt.n_maps * 6), dim3(kReduceBlock), 0, s, j.partials,
                     blocks, ng * 6, j.grad);
  return hipGetLastError();
}

}  // namespace cfs
