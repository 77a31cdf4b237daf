// cfs_batch_dev.hpp -- descriptors and launch arguments of the batched form.
#pragma once

#include <hip/hip_runtime.h>

#include "cfs_params.hpp"

namespace cfs {

constexpr int kClearParts = 16;
// binned FP32 items, binned FP64 items, accumulate items, direct FP32 items,
// direct FP64 items
constexpr int kQueues = 5;

// One instance as the persistent kernels see it (device memory).
struct InstDesc {
  MapTable<2> mt;
  Window win;
  RunArgs ra;
  uint32_t *img;
  unsigned long long *dropped;
  uint32_t elems, n_tiles, flushes, n_chunks;
  uint64_t rec_base;    // first record of the instance's chunks
  uint64_t table_base;  // first word of the instance's run-start tables
  int32_t equal;
  int32_t precision;    // 0 = FP32 positions, 1 = FP64
  uint32_t log2g;       // accumulate lanes per run: 2^log2g
};

struct EmitItem {
  uint32_t inst, first_block, n_blocks;
};

struct AccItem {
  uint32_t inst, tile, c_lo, c_hi;  // chunk range [c_lo, c_hi) of the tile
};

struct TransItem {
  uint32_t inst, bx, by;  // 64x64 block of the instance's table transpose
};

struct BatchLaunch {
  InstDesc *desc;
  uint32_t n_inst;
  const EmitItem *items;  // binned instances: FP32 items, then FP64 items
  uint32_t n_items32, n_items64;
  const EmitItem *ditems;  // direct-splat instances: FP32 items, then FP64 items
  uint32_t n_direct32, n_direct64;
  const AccItem *acc;
  uint32_t n_acc;
  uint32_t *queues;  // [kQueues]
  const TransItem *trans;
  uint32_t n_trans;
  uint16_t *records;
  uint16_t *ctables;  // [chunk][tile + 1] per instance: run starts within the chunk
  uint16_t *tables;   // [tile + 1][chunk] per instance
  uint32_t emit_grid, acc_grid;
};

hipError_t launch_batch(const BatchLaunch &b, hipStream_t stream);
hipError_t launch_batch_set_table(InstDesc *desc, uint32_t index, const MapTable<2> &mt, bool equal,
                                  hipStream_t stream);

}  // namespace cfs
