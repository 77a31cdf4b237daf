// cfs_params.hpp -- kernel-argument structs shared by the host launchers and
// the kernels of the library (plain data, passed by value).
#pragma once

#include <stdint.h>

namespace cfs {

constexpr int kMaxMaps = 64;
// Selection guide: for each of the 2^kGuideBits buckets of the top bits of a
// draw, the range of thresholds that can lie inside the bucket.  The LDS
// threshold array holds kMaxMaps thresholds followed by the guide.
constexpr int kGuideBits = 8;
constexpr int kGuide = 1 << kGuideBits;
constexpr int kThWords = kMaxMaps + kGuide;

constexpr int kFinalIdentity = 0;
constexpr int kFinalSwirl = 1;
constexpr int kFinalTwistCamera = 2;
constexpr int kFinalStretch = 3;
constexpr int kFinalRing = 4;

// Map table of one system: per map A row-major then b (dim*(dim+1) floats),
// and the finite selection thresholds.  n_search == 0 selects with equal
// probabilities; otherwise thresh[0 .. n_search-2] are the thresholds that
// are below 2^32 and the draw picks among the first n_search maps.
// MapTable::flags: some map is a circle map (see circle_mask); the composed
// transform is fed back into the iteration instead of applied to a copy.
constexpr int32_t kFlagCircle = 1;
constexpr int32_t kFlagReuse = 2;

template <int DIM>
struct MapTable {
  float coef[kMaxMaps * DIM * (DIM + 1)];
  uint32_t thresh[kMaxMaps];
  int32_t n_maps;
  int32_t n_search;
  int32_t flags;     // kFlagCircle | kFlagReuse (uniform per system)
  uint64_t circle_mask;  // bit m: map m is a circle map
  int32_t lin;  // kLinGeneral, or every map shares map 0's linear part: kLinShared, kLinScalar
};

// Linear parts of a system's maps: one per map (kLinGeneral); one for all
// maps, bit for bit (kLinShared); one for all maps and a multiple s I of the
// identity (kLinScalar: similarity maps without rotation, such as the
// Sierpinski triangle's, the square's and the Menger sponge's).
constexpr int kLinGeneral = 0;
constexpr int kLinShared = 1;
constexpr int kLinScalar = 2;

// Rows of the translations-only LDS table of a system whose maps share one
// linear part: b of each map, padded to 16-byte reads.
template <int DIM>
struct BRowStride {
  static constexpr int value = (DIM == 2) ? 2 : 4;
};

struct Window {
  int32_t width, height, channels;
  int32_t by_index;  // channel = last map index
  double lo[2];
  double scale[2];   // width / (hi - lo), height / (hi - lo)
};

struct RunArgs {
  uint32_t k0, k1;   // Philox key (seed words)
  uint32_t instance;
  uint32_t n_points;
  uint32_t point_offset;
  uint32_t n_iters;
  uint32_t burn_in;     // steps of this call that are not splatted
  uint32_t iter_block;  // Philox blocks of steps already taken (iter_offset / 4); > 0:
                        // a continued run, started from Outputs::final_points
};

// Binned integer splat: a workgroup of kBinBlock lanes (two per CU fit in
// LDS, so one computes while the other sorts) collects kBinSlots
// splats per lane (one chunk of kChunkCap records), sorts them by image tile
// of kTileElems elements in LDS and writes each tile's records as a run of
// 16-bit in-tile offsets; a per-tile kernel then accumulates the runs in LDS.
constexpr int kBinBlock = 512;
constexpr int kBinSlots = 24;
constexpr uint32_t kChunkCap = static_cast<uint32_t>(kBinBlock) * kBinSlots;
constexpr int kTileBits = 14;
constexpr uint32_t kTileElems = 1u << kTileBits;
constexpr int kMaxTiles = 2048;  // images of up to 2^25 elements
constexpr int kAccBlock = 1024;  // two per CU: 8 waves per SIMD

// Binned depth splat: records are (pixel | index << 24, FP32 depth bits),
// kDSlots per lane per chunk, sorted by tiles of kDTileElems pixels whose
// u64 keys and u32 counts fit in LDS together.  One 1024-lane workgroup per
// CU with a 128 KB stage: 16384 records per chunk, so that each chunk's run
// of a tile is long (the accumulate reads runs scattered over the records,
// and longer runs fetch fewer partly used cache lines); sixteen slots hold a
// run of 16 splatted steps per point in one chunk.
constexpr int kDBlock = 1024;
constexpr int kDSlots = 16;
constexpr uint32_t kDCap = static_cast<uint32_t>(kDBlock) * kDSlots;
constexpr int kDTileBits = 13;
constexpr uint32_t kDTileElems = 1u << kDTileBits;
constexpr int kDAccBlock = 1024;  // one per CU (96 KB of LDS): 4 waves per SIMD

// The depth accumulate's lanes prefetch kDPasses 16-byte loads (two records
// each) per run.  Lanes per run, 2^log2g: the smallest group whose
// prefetch covers a run of the mean length plus one (the even record below
// the start).  The accumulate waits on its scattered loads, and the runs it
// has in flight set its rate: few lanes per run, each with several loads,
// keep the most runs in flight (4 loads of 2 lanes per 15-record run: 3.98
// ms per Menger step; 1 load of 8 lanes: 6.63; 2 loads of 4 lanes: 4.63).
constexpr int kDPasses = 4;
__host__ __device__ inline uint32_t depth_run_lanes_log2(uint64_t mean_run) {
  const uint64_t need = (mean_run + 1u + kDPasses - 1u) / kDPasses;
  uint32_t lg = 0;
  while (lg < 5 && (2ull << lg) < need) ++lg;
  return lg;
}

// The count accumulate aims at this many workgroups (two per CU of MI355X).
constexpr uint32_t kAccTargetGroups = 512;
// ... and at four times as many when it knows the tiles' record totals:
// tiles without records then end at once, so the workgroups that do work
// still fill the chip when much of the image is empty.
constexpr uint32_t kAccTargetSkip = 4 * kAccTargetGroups;

// The count accumulate's lanes prefetch kPasses 16-byte loads (8 records
// each) per run.  Lanes per run, 2^log2g: the smallest group whose prefetch
// covers a run of the mean length plus three (longer runs take further
// loads; larger groups measured slower, and so did 2 or 4 loads per lane
// with smaller groups: 0.44 and 0.52 against 0.42 ms on the CFS square,
// whose two-workgroup-per-CU accumulate already holds many runs in flight).
constexpr int kPasses = 1;
__host__ __device__ inline uint32_t run_lanes_log2(uint64_t mean_run) {
  const uint64_t need = (mean_run + 3u + kPasses - 1u) / kPasses;
  uint32_t lg = 0;
  while (lg < 5 && (8ull << lg) < need) ++lg;
  return lg;
}

struct BinArgs {
  uint16_t *records;     // [n_chunks][kChunkCap] in-tile offsets, runs by tile
  uint2 *drecords;       // depth images: [n_chunks][kDCap] (offset | index << 13, depth)
  uint16_t *chunk_start; // [n_chunks][n_tiles + 1]: run starts within each chunk, as written
  uint16_t *tile_start;  // [n_tiles + 1][n_chunks]: the same, transposed for the accumulate
  uint32_t *tile_sums;   // [n_tiles + 1][n_rb]: column sums of 64-chunk blocks (record totals)
  uint32_t n_rb;         // 64-chunk blocks: ceil(n_chunks / 64)
  uint32_t n_chunks;     // chunks of this launch (= blocks * flushes)
  uint32_t flushes;      // chunks per workgroup
  uint32_t n_tiles;
  uint32_t elems;        // image elements (channels * height * width)
  uint32_t parts;        // accumulate workgroups per tile (chunk ranges)
  uint32_t log2g;        // accumulate lanes per run: 2^log2g
};

// Gaussian splat: 512-lane workgroups collect kGSlots splats per lane as
// (x, y) pixel-coordinate records, sorted by 32x32-pixel tile.  8 slots (a
// 32 KB stage, so that LDS leaves room for three workgroups per CU)
// measured faster than 12 and 16.
constexpr int kGBlock = 512;
constexpr int kGSlots = 8;
constexpr uint32_t kGCap = static_cast<uint32_t>(kGBlock) * kGSlots;
constexpr int kGTileLog = 5;
constexpr int kGTile = 1 << kGTileLog;
constexpr int kGMaxTiles = 2048;
constexpr int kGAccBlock = 256;
// Per-tile Gaussian kernels: at most this many workgroups per tile, each
// taking an equal share of the chunks; a tile uses as many of them as its
// record total asks for at one workgroup per 1/kGPartTarget of the launch's
// splats (small workgroups: the dense tiles' parts then balance over the
// chip; 4096 and 16384 measured slower).
constexpr uint32_t kGMaxParts = 64;
constexpr uint32_t kGPartTarget = 32768;
constexpr int kGBwdBlock = 256;
constexpr int kMaxSeg = 16;  // longest checkpoint segment
constexpr int kShortSeg = 8;  // segments up to this take the lighter adjoint kernel

struct GaussParams {
  float sigma, inv2s2, inv_s2, cutoff, R;  // R = 3 sigma, cutoff = exp(-R^2/2s^2)
  float weight;                            // 1 / (N (T - B)) of the whole run
  int32_t taps;                            // candidate taps per axis
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  float lo[2], scale[2];
};

struct GaussBin {
  float2 *records;       // [n_chunks][kGCap] pixel coordinates, runs by tile
  uint32_t *pos;         // backward only: [T - B][points] each splat's record index, or ~0u
  uint32_t *chunk_start; // [n_chunks][n_tiles + 1] as the chunks write them
  uint32_t *tile_start;  // [n_tiles + 1][n_chunks] transposed for the accumulate
  uint32_t *tile_sums;   // [n_tiles + 1][n_rb]: column sums of 64-chunk blocks (record totals)
  uint32_t n_chunks, flushes, n_tiles, n_rb;
};

struct GaussCkpt {
  float *ckpt;           // [n_ckpt][stride][2] (base already offset to the slice)
  int32_t every;
  uint32_t stride;       // points of the whole run
};

// Objects of a scene (several objects from one primitive): transform kind
// and its first 8 parameters, placement, channel and duplication.
constexpr int kMaxObjects = 8;
// Copies of duplicated objects whose placements a scene workgroup keeps in
// LDS (filled once per workgroup from the same random streams; objects past
// this budget draw each copy's placement per splat).
constexpr uint32_t kSceneCopyTable = 512;

struct SceneObject {
  int32_t kind;
  int32_t channel;
  uint32_t n_copies;
  int32_t tab_base;  // first LDS placement row of this object's copies, or -1
  float fp[8];
  float place[6];
  float copy_lo[2], copy_span[2];
  float scale_lo, scale_span;
};
struct SceneArgs {
  SceneObject obj[kMaxObjects];
  int32_t n_obj;
  int32_t any_copies;
};

struct Outputs {
  void *final_points;          // float or double [N][dim], nullable
  uint8_t *last_index;         // [N], nullable
  uint8_t *indices;            // [N][T], nullable
  unsigned long long *dropped; // nullable
};

}  // namespace cfs
