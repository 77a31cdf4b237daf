// k_batch.hip -- batched chaos game: many heterogeneous instances rendered by
// persistent workgroups that pop work items from a device queue.
//
// An instance is one 2D affine system with its run and image.  Emit items are
// (instance, first 512-point block, block count); accumulate items are
// (instance, image tile, chunk range).  Each instance takes the binned or
// the direct splat, as the plan's per-instance threshold says.  Each item loads its instance's descriptor (map
// table and thresholds into LDS) and runs exactly the device functions of a
// plain run, so every instance's image is bit-identical to cfs_chaos_game's.
// The queues hold a known number of items and every workgroup leaves when a
// pop returns an index past the end, so the grids always drain.
#include "cfs_batch_dev.hpp"
#include "cfs_binned.hpp"
#include "cfs_direct.hpp"

namespace cfs {

// Pop the next item index (one atomic per item, broadcast through LDS).
__device__ __forceinline__ uint32_t pop_item(uint32_t *queue, uint32_t *slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(queue, 1u);
  __syncthreads();
  // the same value in every lane: keep it (and the item and descriptor loads
  // indexed by it) on the scalar unit
  const uint32_t it = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();
  return it;
}

// Persistent chaos kernel for the instances of one position type.
template <typename real>
__global__ __launch_bounds__(kBinBlock) void k_batch_emit(const InstDesc *__restrict__ desc,
                                                          const EmitItem *__restrict__ items,
                                                          uint32_t n_items, uint32_t *queue,
                                                          uint16_t *records, uint16_t *ctables,
                                                          uint16_t *tables) {
  __shared__ real table[kMaxMaps * RowStride<real, 2>::value];
  __shared__ uint32_t th[kThWords];
  __shared__ uint32_t stage[kChunkCap];
  __shared__ uint32_t cnt[kMaxTiles];
  __shared__ uint32_t wsum[kWaves + 1];
  __shared__ uint32_t slot;
  for (uint32_t t = threadIdx.x; t < kMaxTiles; t += kBinBlock) cnt[t] = 0u;
  __syncthreads();
  for (;;) {
    const uint32_t it = pop_item(queue, &slot);
    if (it >= n_items) break;
    const EmitItem item = items[it];
    const InstDesc &d = desc[item.inst];
    load_table<real, 2, false>(d.mt, table, th);
    __syncthreads();
    // the item's descriptor fields as values (uniform, so they stay in
    // scalar registers instead of being reloaded inside the point loop)
    const Window win = d.win;
    const RunArgs ra = d.ra;
    const int n_maps = d.mt.n_maps, n_search = d.mt.n_search, flags = d.mt.flags;
    BinArgs ba;
    ba.records = records + d.rec_base;
    ba.chunk_start = ctables + d.table_base;
    ba.tile_start = tables + d.table_base;
    ba.n_chunks = d.n_chunks;
    ba.flushes = d.flushes;
    ba.n_tiles = d.n_tiles;
    ba.elems = d.elems;
    Outputs out{nullptr, nullptr, nullptr, d.dropped};
    for (uint32_t b = 0; b < item.n_blocks; ++b)
      chaos_binned_block<real, 2, kFinalIdentity, kSelRuntime, false>(
          table, th, n_maps, n_search, flags, win, ra, nullptr, ba, out, item.first_block + b,
          stage, cnt, wsum);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kAccBlock) void k_batch_accumulate(const InstDesc *__restrict__ desc,
                                                                const AccItem *__restrict__ items,
                                                                uint32_t n_items, uint32_t *queue,
                                                                const uint16_t *records,
                                                                const uint16_t *tables) {
  __shared__ uint32_t tile[kTileElems];
  __shared__ uint32_t slot;
  for (;;) {
    const uint32_t it = pop_item(queue, &slot);
    if (it >= n_items) break;
    const AccItem item = items[it];
    const InstDesc &d = desc[item.inst];
    tile_accumulate(records + d.rec_base, tables + d.table_base, d.n_chunks, item.c_lo, item.c_hi,
                    d.elems, d.img, item.tile, d.log2g, tile);
  }
}

// Transpose every instance's [chunk][tile] run-start table into [tile][chunk]
// (one 64x64 block per workgroup).
__global__ __launch_bounds__(256) void k_batch_transpose(const InstDesc *__restrict__ desc,
                                                         const TransItem *__restrict__ items,
                                                         const uint16_t *ctables, uint16_t *tables) {
  __shared__ uint32_t buf[64][65];
  const TransItem it = items[blockIdx.x];
  const InstDesc &d = desc[it.inst];
  transpose_tile(ctables + d.table_base, tables + d.table_base, d.n_chunks, d.n_tiles + 1, it.bx,
                 it.by, buf);
}

// Direct splat: the same per-point function as the plain direct kernel.
template <typename real>
__global__ __launch_bounds__(kBinBlock) void k_batch_direct(const InstDesc *__restrict__ desc,
                                                            const EmitItem *__restrict__ items,
                                                            uint32_t n_items, uint32_t *queue) {
  __shared__ real table[kMaxMaps * RowStride<real, 2>::value];
  __shared__ uint32_t th[kThWords];
  __shared__ uint32_t slot;
  for (;;) {
    const uint32_t it = pop_item(queue, &slot);
    if (it >= n_items) break;
    const EmitItem item = items[it];
    const InstDesc &d = desc[item.inst];
    load_table<real, 2, false>(d.mt, table, th);
    __syncthreads();
    const Window win = d.win;
    const RunArgs ra = d.ra;
    const int n_maps = d.mt.n_maps, n_search = d.mt.n_search, flags = d.mt.flags;
    uint32_t *img = d.img;
    Outputs out{nullptr, nullptr, nullptr, d.dropped};
    for (uint32_t b = 0; b < item.n_blocks; ++b)
      chaos_direct_point<real, 2, kFinalIdentity, kSelRuntime, false, false>(
          table, th, n_maps, n_search, flags, win, ra, nullptr, img, nullptr, 0.0f, out,
          (item.first_block + b) * kBinBlock + threadIdx.x);
    __syncthreads();
  }
}

// Clear every image (kClearParts workgroups per instance), zero the dropped
// counters and reset every queue.  Plain stores only (graph-safe).
__global__ void k_batch_clear(const InstDesc *__restrict__ desc, uint32_t n_inst, uint32_t *queues) {
  const uint32_t inst = blockIdx.x / kClearParts;
  const uint32_t part = blockIdx.x % kClearParts;
  if (blockIdx.x == 0 && threadIdx.x < kQueues) queues[threadIdx.x] = 0u;
  if (inst >= n_inst) return;
  const InstDesc &d = desc[inst];
  const size_t per = (static_cast<size_t>(d.elems) + kClearParts - 1) / kClearParts;
  const size_t lo = part * per;
  const size_t hi = min(static_cast<size_t>(d.elems), lo + per);
  for (size_t i = lo + threadIdx.x; i < hi; i += blockDim.x) d.img[i] = 0u;
  if (part == 0 && threadIdx.x == 0 && d.dropped) *d.dropped = 0ull;
}

__global__ void k_batch_set_table(InstDesc *desc, uint32_t index, MapTable<2> mt, int32_t equal) {
  // one thread copies the new table (stream-ordered, no host buffer involved)
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    desc[index].mt = mt;
    desc[index].equal = equal;
  }
}

hipError_t launch_batch(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_clear, dim3(b.n_inst * kClearParts), dim3(256), 0, s, b.desc, b.n_inst,
                     b.queues);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // binned instances (FP32 then FP64, each from its own queue), then the
  // direct-splat instances, then the binned instances' transposes and tiles
  if (b.n_items32)
    hipLaunchKernelGGL(k_batch_emit<float>, dim3(b.emit_grid), dim3(kBinBlock), 0, s, b.desc, b.items,
                       b.n_items32, b.queues + 0, b.records, b.ctables, b.tables);
  if (b.n_items64)
    hipLaunchKernelGGL(k_batch_emit<double>, dim3(b.emit_grid), dim3(kBinBlock), 0, s, b.desc,
                       b.items + b.n_items32, b.n_items64, b.queues + 1, b.records, b.ctables,
                       b.tables);
  if (b.n_direct32)
    hipLaunchKernelGGL(k_batch_direct<float>, dim3(b.emit_grid), dim3(kBinBlock), 0, s, b.desc,
                       b.ditems, b.n_direct32, b.queues + 3);
  if (b.n_direct64)
    hipLaunchKernelGGL(k_batch_direct<double>, dim3(b.emit_grid), dim3(kBinBlock), 0, s, b.desc,
                       b.ditems + b.n_direct32, b.n_direct64, b.queues + 4);
  if (b.n_trans)
    hipLaunchKernelGGL(k_batch_transpose, dim3(b.n_trans), dim3(256), 0, s, b.desc, b.trans,
                       b.ctables, b.tables);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b.n_acc)
    hipLaunchKernelGGL(k_batch_accumulate, dim3(b.acc_grid), dim3(kAccBlock), 0, s, b.desc, b.acc,
                       b.n_acc, b.queues + 2, b.records, b.tables);
  return hipGetLastError();
}

hipError_t launch_batch_set_table(InstDesc *desc, uint32_t index, const MapTable<2> &mt, bool equal,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_batch_set_table, dim3(1), dim3(64), 0, s, desc, index, mt, equal ? 1 : 0);
  return hipGetLastError();
}

}  // namespace cfs
