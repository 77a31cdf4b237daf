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
#include "cfs_binned.hpp"
#include "cfs_host.hpp"

namespace cfs {

template <typename real, int DIM, int FINAL, bool EQUAL, bool GENERAL, int LIN>
__global__ __launch_bounds__(kBinBlock) void k_chaos_binned(MapTable<DIM> mt, Window win,
                                                            RunArgs ra, FinalArgs fa, BinArgs ba,
                                                            Outputs out) {
  __shared__ real table[kMaxMaps * RowStride<real, DIM>::value];
  __shared__ uint32_t th[kThWords];
  __shared__ uint32_t stage[kChunkCap];
  __shared__ uint32_t cnt[kMaxTiles];
  __shared__ uint32_t wsum[kWaves + 1];
  load_table<real, DIM, sizeof(real) == sizeof(double), LIN != kLinGeneral>(mt, table, th);
  for (uint32_t t = threadIdx.x; t < ba.n_tiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();
  chaos_binned_block<real, DIM, FINAL, EQUAL, GENERAL, LIN>(
      table, th, mt.n_maps, mt.n_search, mt.flags, win, ra, fa.p, ba, out, blockIdx.x, stage, cnt,
      wsum, shared_linear<real, DIM>(mt));
}

// The map table sits in dynamic LDS sized for the system's own maps, so that
// the 64 KB stage leaves room for two workgroups per CU.
// One 1024-lane workgroup per CU (the 128 KB stage): four waves per SIMD,
// 128 VGPRs.
template <typename real, bool EQUAL, int LIN>
__global__ __launch_bounds__(kDBlock) void k_chaos_depth_binned(MapTable<3> mt, Window win,
                                                                  RunArgs ra, FinalArgs fa,
                                                                  float near_plane, BinArgs ba,
                                                                  Outputs out) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  real *table = reinterpret_cast<real *>(dyn_lds);
  __shared__ uint32_t th[kThWords];
  __shared__ uint2 stage[kDCap];
  __shared__ uint32_t cnt[kMaxTiles];
  __shared__ uint32_t wsum[kDWaves + 1];
  __shared__ real fparams[kFinalParams];
  load_table<real, 3, sizeof(real) == sizeof(double), LIN != kLinGeneral>(mt, table, th);
  for (uint32_t t = threadIdx.x; t < ba.n_tiles; t += kDBlock) cnt[t] = 0u;
  if (threadIdx.x < kFinalParams) fparams[threadIdx.x] = static_cast<real>(fa.p[threadIdx.x]);
  __syncthreads();
  chaos_depth_block<real, EQUAL ? kSelEqual : kSelTable, LIN>(
      table, th, mt.n_maps, mt.n_search, win, ra, fparams, near_plane, ba, out, blockIdx.x, stage,
      cnt, wsum, shared_linear<real, 3>(mt));
}

// Record total of tile t over all chunks, from the transpose's column sums
// of 64-chunk blocks (every thread of the workgroup calls it and gets it).
__device__ inline uint32_t tile_total(const uint32_t *__restrict__ sums, uint32_t n_rb, uint32_t t,
                                      uint32_t *red) {
  const uint32_t tid = threadIdx.x;
  const uint32_t *lo = sums + static_cast<size_t>(t) * n_rb, *hi = lo + n_rb;
  uint32_t s = 0;
  for (uint32_t b = tid; b < n_rb; b += kAccBlock) s += hi[b] - lo[b];
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  uint32_t total = 0;
#pragma unroll
  for (int w = 0; w < kAccBlock / 64; ++w) total += red[w];
  return total;
}

// One workgroup per depth tile, taken in XCD-contiguous order (the runs of
// neighbouring tiles share cache lines in every chunk); a tile without
// records (from the transpose's column sums) ends at once, and the lanes per
// run follow the tile's own mean run length.
__global__ __launch_bounds__(kDAccBlock) void k_depth_accumulate(const uint2 *__restrict__ rec,
                                                                 const uint16_t *__restrict__ tile_start,
                                                                 const uint32_t *__restrict__ sums,
                                                                 uint32_t n_rb, uint32_t n_chunks,
                                                                 uint32_t elems,
                                                                 unsigned long long *img,
                                                                 uint32_t *density) {
  __shared__ unsigned long long keys[kDTileElems];
  __shared__ uint32_t counts[kDTileElems];
  __shared__ uint32_t red[kDAccBlock / 64];
  static_assert(kDAccBlock == kAccBlock, "tile_total sums over kAccBlock lanes");
  const uint32_t t = xcd_item(blockIdx.x, gridDim.x);
  const uint32_t total = tile_total(sums, n_rb, t, red);
  if (total == 0) return;  // the same value in every lane
  depth_tile_accumulate(rec, tile_start, n_chunks, elems, img, density, t,
                        depth_run_lanes_log2(total / n_chunks), keys, counts);
}

// One workgroup per (image tile, chunk range); the parts of a tile are
// neighbours in the XCD-contiguous order.  With the tiles' record totals
// (`sums`), a tile without records is skipped and each tile walks its runs
// with the lane group that its own mean run length asks for; without them,
// every tile uses `log2g`.
__global__ __launch_bounds__(kAccBlock) void k_tile_accumulate(const uint16_t *__restrict__ rec,
                                                               const uint16_t *__restrict__ tile_start,
                                                               const uint32_t *__restrict__ sums,
                                                               uint32_t n_rb, uint32_t n_chunks,
                                                               uint32_t elems,
                                                               uint32_t *__restrict__ img,
                                                               uint32_t parts, uint32_t log2g) {
  __shared__ uint32_t tile[kTileElems];
  __shared__ uint32_t red[kAccBlock / 64];
  const uint32_t item = xcd_item(blockIdx.x, gridDim.x);
  const uint32_t t = item / parts, part = item % parts;
  if (sums) {
    const uint32_t total = tile_total(sums, n_rb, t, red);
    if (total == 0) return;  // the same value in every lane
    log2g = run_lanes_log2(total / n_chunks);
  }
  const uint32_t c_lo = static_cast<uint32_t>(static_cast<uint64_t>(n_chunks) * part / parts);
  const uint32_t c_hi = static_cast<uint32_t>(static_cast<uint64_t>(n_chunks) * (part + 1) / parts);
  tile_accumulate(rec, tile_start, n_chunks, c_lo, c_hi, elems, img, t, log2g, tile);
}

template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ in, T *__restrict__ out,
                                                    uint32_t rows, uint32_t cols,
                                                    uint32_t *__restrict__ sums) {
  __shared__ uint32_t buf[64][65];
  transpose_tile(in, out, rows, cols, blockIdx.x, blockIdx.y, buf, sums, gridDim.y);
}

template <typename T>
static hipError_t launch_transpose_t(const T *in, T *out, uint32_t rows, uint32_t cols,
                                     hipStream_t s, uint32_t *sums) {
  if (rows == 0 || cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose<T>, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s, in,
                     out, rows, cols, sums);
  return hipGetLastError();
}

hipError_t launch_transpose(const uint32_t *in, uint32_t *out, uint32_t rows, uint32_t cols,
                            hipStream_t s, uint32_t *sums) {
  return launch_transpose_t(in, out, rows, cols, s, sums);
}

hipError_t launch_transpose(const uint16_t *in, uint16_t *out, uint32_t rows, uint32_t cols,
                            hipStream_t s, uint32_t *sums) {
  return launch_transpose_t(in, out, rows, cols, s, sums);
}

void acc_shape(uint64_t records, uint32_t n_chunks, uint32_t n_tiles, uint32_t target,
               uint32_t *parts, uint32_t *log2g) {
  // mean run length -> lanes per run (a lane loads 8 records)
  const uint64_t runs = static_cast<uint64_t>(n_chunks) * (n_tiles ? n_tiles : 1);
  const uint64_t mean = runs ? records / runs : 0;
  uint32_t lg = 0;
  while (lg < 5 && (8ull << lg) < mean) ++lg;
  *log2g = lg;
  // about `target` workgroups, but at least one pass of groups each
  const uint32_t groups = kAccBlock >> lg;
  uint32_t p = n_tiles ? (target + n_tiles - 1) / n_tiles : 1;
  const uint32_t pmax = n_chunks / groups > 1 ? n_chunks / groups : 1;
  *parts = p < 1 ? 1 : (p > pmax ? pmax : p);
}

BinPlan bin_plan(uint32_t points, uint32_t n_iters, uint32_t burn_in, uint32_t elems, bool depth,
                 uint32_t per_iter) {
  BinPlan bp{};
  const uint32_t slots = depth ? kDSlots : kBinSlots;
  const uint32_t block = depth ? kDBlock : kBinBlock;
  bp.blocks = (points + block - 1) / block;
  bp.flushes = ((n_iters - burn_in) * per_iter + slots - 1) / slots;
  bp.n_chunks = bp.blocks * bp.flushes;
  bp.n_tiles = depth ? (elems + kDTileElems - 1) / kDTileElems : (elems + kTileElems - 1) / kTileElems;
  bp.elems = elems;
  acc_shape(static_cast<uint64_t>(points) * (n_iters - burn_in) * per_iter, bp.n_chunks, bp.n_tiles,
            kAccTargetSkip, &bp.parts, &bp.log2g);
  bp.records_bytes = depth ? static_cast<size_t>(bp.n_chunks) * kDCap * sizeof(uint2)
                           : static_cast<size_t>(bp.n_chunks) * kChunkCap * sizeof(uint16_t);
  bp.table_bytes = static_cast<size_t>(bp.n_tiles + 1) * bp.n_chunks * sizeof(uint16_t);  // each of two
  bp.n_rb = (bp.n_chunks + 63) / 64;
  bp.sums_bytes = static_cast<size_t>(bp.n_tiles + 1) * bp.n_rb * sizeof(uint32_t);
  return bp;
}

hipError_t launch_count_accumulate(const BinArgs &ba, uint32_t *img, hipStream_t s,
                                   const hipEvent_t *ev) {
  hipError_t e = launch_transpose(ba.chunk_start, ba.tile_start, ba.n_chunks, ba.n_tiles + 1, s,
                                  ba.tile_sums);
  if (e != hipSuccess) return e;
  mark_phase(ev, 2, s);
  hipLaunchKernelGGL(k_tile_accumulate, dim3(ba.n_tiles * ba.parts), dim3(kAccBlock), 0, s,
                     ba.records, ba.tile_start, ba.tile_sums, ba.n_rb, ba.n_chunks, ba.elems, img,
                     ba.parts, ba.log2g);
  e = hipGetLastError();
  mark_phase(ev, 3, s);
  return e;
}

template <typename real, int DIM, int FINAL, bool EQUAL>
static hipError_t launch_binned_typed(const ChaosJob &j, hipStream_t s) {
  const MapTable<DIM> &mt = [&]() -> const MapTable<DIM> & {
    if constexpr (DIM == 2) return j.mt2; else return j.mt3;
  }();
  const uint32_t blocks = (j.ra.n_points + kBinBlock - 1) / kBinBlock;
  mark_phase(j.ev, 0, s);
  // circle maps, reuse composition (2D only) and continued runs take the
  // general variant; systems whose maps share one linear part gather only
  // the translations
  if (mt.flags != 0 || j.ra.iter_block != 0)
    hipLaunchKernelGGL((k_chaos_binned<real, DIM, FINAL, EQUAL, true, kLinGeneral>), dim3(blocks),
                       dim3(kBinBlock), 0, s, mt, j.win, j.ra, j.fa, j.ba, j.out);
  else if (mt.lin == kLinScalar)
    hipLaunchKernelGGL((k_chaos_binned<real, DIM, FINAL, EQUAL, false, kLinScalar>), dim3(blocks),
                       dim3(kBinBlock), 0, s, mt, j.win, j.ra, j.fa, j.ba, j.out);
  else if (mt.lin == kLinShared)
    hipLaunchKernelGGL((k_chaos_binned<real, DIM, FINAL, EQUAL, false, kLinShared>), dim3(blocks),
                       dim3(kBinBlock), 0, s, mt, j.win, j.ra, j.fa, j.ba, j.out);
  else
    hipLaunchKernelGGL((k_chaos_binned<real, DIM, FINAL, EQUAL, false, kLinGeneral>), dim3(blocks),
                       dim3(kBinBlock), 0, s, mt, j.win, j.ra, j.fa, j.ba, j.out);
  hipError_t e = hipGetLastError();
  mark_phase(j.ev, 1, s);
  if (e != hipSuccess) return e;
  if (j.ba.n_chunks == 0) {
    mark_phase(j.ev, 2, s);
    mark_phase(j.ev, 3, s);
    return e;
  }
  return launch_count_accumulate(j.ba, static_cast<uint32_t *>(j.img), s, j.ev);
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
    case kFinalRing: return launch_binned_sel<real, 2, kFinalRing>(j, s);
    default: return launch_binned_sel<real, 2, kFinalIdentity>(j, s);
  }
}

template <typename real>
static hipError_t launch_depth_binned(const ChaosJob &j, hipStream_t s) {
  const uint32_t blocks = (j.ra.n_points + kDBlock - 1) / kDBlock;
  const int lin = j.mt3.lin;
  const size_t table_bytes =
      static_cast<size_t>(j.mt3.n_maps) *
      (lin != kLinGeneral ? BRowStride<3>::value : RowStride<real, 3>::value) * sizeof(real);
  mark_phase(j.ev, 0, s);
#define CFS_DEPTH_LAUNCH(EQ, LN)                                                               \
  hipLaunchKernelGGL((k_chaos_depth_binned<real, EQ, LN>), dim3(blocks), dim3(kDBlock),        \
                     table_bytes, s, j.mt3, j.win, j.ra, j.fa, j.near_plane, j.ba, j.out)
  if (j.equal) {
    if (lin == kLinScalar) CFS_DEPTH_LAUNCH(true, kLinScalar);
    else if (lin == kLinShared) CFS_DEPTH_LAUNCH(true, kLinShared);
    else CFS_DEPTH_LAUNCH(true, kLinGeneral);
  } else {
    if (lin == kLinScalar) CFS_DEPTH_LAUNCH(false, kLinScalar);
    else if (lin == kLinShared) CFS_DEPTH_LAUNCH(false, kLinShared);
    else CFS_DEPTH_LAUNCH(false, kLinGeneral);
  }
#undef CFS_DEPTH_LAUNCH
  hipError_t e = hipGetLastError();
  mark_phase(j.ev, 1, s);
  if (e == hipSuccess && j.ba.n_chunks != 0)
    e = launch_transpose(j.ba.chunk_start, j.ba.tile_start, j.ba.n_chunks, j.ba.n_tiles + 1, s,
                         j.ba.tile_sums);
  mark_phase(j.ev, 2, s);
  if (e == hipSuccess && j.ba.n_chunks != 0) {
    hipLaunchKernelGGL(k_depth_accumulate, dim3(j.ba.n_tiles), dim3(kDAccBlock), 0, s,
                       j.ba.drecords, j.ba.tile_start, j.ba.tile_sums, j.ba.n_rb, j.ba.n_chunks,
                       j.ba.elems, static_cast<unsigned long long *>(j.img), j.density);
    e = hipGetLastError();
  }
  mark_phase(j.ev, 3, s);
  return e;
}

hipError_t launch_chaos_binned(const ChaosJob &job, hipStream_t stream) {
  if (job.ra.n_points == 0) {
    for (int i = 0; i < kPhaseEvents; ++i) mark_phase(job.ev, i, stream);
    return hipSuccess;
  }
  if (job.depth)
    return job.precision == 1 ? launch_depth_binned<double>(job, stream)
                              : launch_depth_binned<float>(job, stream);
  return job.precision == 1 ? launch_binned_real<double>(job, stream)
                            : launch_binned_real<float>(job, stream);
}

}  // namespace cfs
