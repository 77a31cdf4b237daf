// cfs_api_batch.hip -- C ABI of the batched form: batch construction (device
// descriptors, work queues, records), HIP-graph capture and replay, per-frame
// updates, and the autotuner that picks a schedule by timing graph replays.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cfs.h"
#include "cfs_api_internal.hpp"
#include "cfs_batch_dev.hpp"
#include "cfs_host.hpp"

using namespace cfs;

struct cfs_batch {
  int device = -1;
  int32_t n = 0;
  cfs_plan plan{};
  int cus = 0;
  InstDesc *d_desc = nullptr;
  EmitItem *d_items = nullptr;
  AccItem *d_acc = nullptr;
  TransItem *d_trans = nullptr;
  uint16_t *d_ctables = nullptr;
  uint32_t *d_queues = nullptr;
  uint16_t *d_records = nullptr;
  uint16_t *d_tables = nullptr;
  uint32_t n_items32 = 0, n_items64 = 0, n_direct32 = 0, n_direct64 = 0, n_acc = 0, n_trans = 0;
  std::vector<int32_t> n_maps;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(cfs_batch *b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->capture_stream) hipStreamDestroy(b->capture_stream);
  hipFree(b->d_desc);
  hipFree(b->d_items);
  hipFree(b->d_acc);
  hipFree(b->d_trans);
  hipFree(b->d_ctables);
  hipFree(b->d_queues);
  hipFree(b->d_records);
  hipFree(b->d_tables);
  delete b;
}

int validate_item(const cfs_batch_item &it, int i) {
  int rc = validate_system(&it.sys);
  if (!rc) rc = validate_fresh_run(&it.run);
  if (!rc) rc = validate_window(&it.img);
  if (rc) return fail(rc, "batch item %d: %s", i, cfs_last_error());
  if (it.sys.dim != 2 || it.sys.final_kind != CFS_FINAL_IDENTITY)
    return fail(CFS_E_UNSUPPORTED, "batch item %d: 2D systems with the identity transform only", i);
  if (it.sys.kind)
    for (int m = 0; m < it.sys.n_maps; ++m)
      if (it.sys.kind[m] != CFS_MAP_AFFINE)
        return fail(CFS_E_UNSUPPORTED, "batch item %d: affine maps only", i);
  if (it.img.kind != CFS_IMAGE_U32_COUNT ||
      (it.img.channels != 1 && it.img.channels != it.sys.n_maps))
    return fail(CFS_E_INVALID, "batch item %d: U32_COUNT image with 1 or n_maps channels", i);
  const uint64_t elems = static_cast<uint64_t>(it.img.width) * it.img.height * it.img.channels;
  if (elems > static_cast<uint64_t>(kMaxTiles) * kTileElems)
    return fail(CFS_E_UNSUPPORTED, "batch item %d: image larger than %u elements", i,
                static_cast<unsigned>(kMaxTiles * kTileElems));
  const uint64_t blocks = (it.run.n_points + kBinBlock - 1) / kBinBlock;
  const uint64_t flushes = (it.run.n_iters - it.run.burn_in + kBinSlots - 1) / kBinSlots;
  if (blocks * flushes * kChunkCap >= (1ull << 31))
    return fail(CFS_E_UNSUPPORTED, "batch item %d: too many splats for one instance", i);
  return CFS_OK;
}

int normalise_plan(const cfs_plan *in, int cus, cfs_plan *out) {
  // default: four blocks per item (256 random systems: 7.59 ms per graph
  // launch against 7.76 with one; the accumulate grid barely matters)
  cfs_plan p{4, 0, 0, CFS_SPLAT_BINNED, 0};
  if (in) p = *in;
  if (p.blocks_per_item < 1 || p.blocks_per_item > 1024)
    return fail(CFS_E_INVALID, "plan.blocks_per_item must be in 1..1024");
  if (p.emit_grid < 0 || p.acc_grid < 0) return fail(CFS_E_INVALID, "plan grids must be >= 0");
  if (p.splat_path == CFS_SPLAT_AUTO) p.splat_path = CFS_SPLAT_BINNED;
  if (p.splat_path != CFS_SPLAT_BINNED && p.splat_path != CFS_SPLAT_DIRECT)
    return fail(CFS_E_INVALID, "plan.splat_path must be BINNED or DIRECT");
  if (p.emit_grid == 0) p.emit_grid = 2 * cus;
  if (p.acc_grid == 0) p.acc_grid = 2 * cus;
  *out = p;
  return CFS_OK;
}

#define HIP_TRY(call, what)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) {                                   \
      int rc_ = device_status(e_, what);                      \
      free_batch(b);                                          \
      return rc_ == CFS_OK ? CFS_E_DEVICE : rc_;              \
    }                                                         \
  } while (0)

}  // namespace

extern "C" int cfs_batch_create(const cfs_batch_item *items, int32_t n_items, const cfs_plan *plan,
                                cfs_batch **out) {
  clear_error();
  if (!out) return fail(CFS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!items || n_items < 1) return fail(CFS_E_INVALID, "need at least one batch item");
  for (int i = 0; i < n_items; ++i) {
    const int rc = validate_item(items[i], i);
    if (rc) return rc;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return device_status(e, "hipDeviceGetAttribute");
  cfs_plan p;
  int rc = normalise_plan(plan, cus, &p);
  if (rc) return rc;

  std::vector<InstDesc> desc(n_items);
  std::vector<EmitItem> emit, direct;
  std::vector<AccItem> acc;
  std::vector<TransItem> trans;
  uint64_t rec_total = 0, table_total = 0;
  for (int i = 0; i < n_items; ++i) {
    const cfs_batch_item &it = items[i];
    InstDesc &d = desc[i];
    std::memset(&d, 0, sizeof d);
    bool equal = false;
    rc = pack_table<2>(&it.sys, &d.mt, &equal);
    if (rc) return rc;
    d.equal = equal ? 1 : 0;
    d.precision = it.run.precision == CFS_PREC_F64 ? 1 : 0;
    d.win = make_window(&it.img, it.img.channels > 1);
    d.ra = make_run_args(&it.run);
    d.img = static_cast<uint32_t *>(it.img.data);
    d.dropped = it.img.dropped;
    d.elems = static_cast<uint32_t>(it.img.width) * it.img.height * it.img.channels;
    const BinPlan bp = bin_plan(it.run.n_points, it.run.n_iters, it.run.burn_in, d.elems);
    // the plan's per-instance strategy: the direct splat for the whole batch,
    // or for the instances with fewer splats than direct_below
    const uint64_t n_splats =
        static_cast<uint64_t>(it.run.n_points) * (it.run.n_iters - it.run.burn_in);
    if (p.splat_path == CFS_SPLAT_DIRECT || n_splats < p.direct_below) {
      d.n_tiles = bp.n_tiles;
      for (uint32_t blk = 0; blk < bp.blocks; blk += p.blocks_per_item)
        direct.push_back(EmitItem{static_cast<uint32_t>(i), blk,
                                  std::min<uint32_t>(p.blocks_per_item, bp.blocks - blk)});
      continue;
    }
    const bool splats = it.run.n_iters > it.run.burn_in;
    d.n_tiles = bp.n_tiles;
    d.flushes = splats ? bp.flushes : 0;
    d.n_chunks = splats ? bp.n_chunks : 0;
    d.rec_base = rec_total;
    d.table_base = table_total;
    rec_total += static_cast<uint64_t>(d.n_chunks) * kChunkCap;
    rec_total = (rec_total + 127) & ~static_cast<uint64_t>(127);
    table_total += static_cast<uint64_t>(d.n_tiles + 1) * d.n_chunks;
    for (uint32_t blk = 0; blk < bp.blocks; blk += p.blocks_per_item)
      emit.push_back(EmitItem{static_cast<uint32_t>(i), blk,
                              std::min<uint32_t>(p.blocks_per_item, bp.blocks - blk)});
    // the batched accumulate walks every tile, so it aims at fewer workgroups
    uint32_t parts = 1;
    acc_shape(static_cast<uint64_t>(it.run.n_points) * (it.run.n_iters - it.run.burn_in),
              bp.n_chunks, bp.n_tiles, kAccTargetGroups, &parts, &d.log2g);
    if (d.n_chunks) {
      for (uint32_t t = 0; t < d.n_tiles; ++t)
        for (uint32_t q = 0; q < parts; ++q)
          acc.push_back(AccItem{static_cast<uint32_t>(i), t,
                                static_cast<uint32_t>(static_cast<uint64_t>(d.n_chunks) * q / parts),
                                static_cast<uint32_t>(static_cast<uint64_t>(d.n_chunks) * (q + 1) / parts)});
      for (uint32_t by = 0; by < (d.n_chunks + 63) / 64; ++by)
        for (uint32_t bx = 0; bx < (d.n_tiles + 1 + 63) / 64; ++bx)
          trans.push_back(TransItem{static_cast<uint32_t>(i), bx, by});
    }
  }
  // FP32 instances' items first, then FP64 ones; within each, largest
  // instances first so the tail of each queue holds small items
  std::stable_sort(emit.begin(), emit.end(), [&](const EmitItem &a, const EmitItem &b2) {
    const InstDesc &da = desc[a.inst], &db = desc[b2.inst];
    if (da.precision != db.precision) return da.precision < db.precision;
    return da.ra.n_points > db.ra.n_points;
  });
  uint32_t n32 = 0;
  for (const EmitItem &it : emit) n32 += desc[it.inst].precision == 0 ? 1u : 0u;
  std::stable_sort(direct.begin(), direct.end(), [&](const EmitItem &a, const EmitItem &b2) {
    const InstDesc &da = desc[a.inst], &db = desc[b2.inst];
    if (da.precision != db.precision) return da.precision < db.precision;
    return da.ra.n_points > db.ra.n_points;
  });
  uint32_t d32 = 0;
  for (const EmitItem &it : direct) d32 += desc[it.inst].precision == 0 ? 1u : 0u;
  // accumulate items by expected record count, largest first
  std::stable_sort(acc.begin(), acc.end(), [&](const AccItem &a, const AccItem &b2) {
    const double wa = static_cast<double>(a.c_hi - a.c_lo) / desc[a.inst].n_tiles;
    const double wb = static_cast<double>(b2.c_hi - b2.c_lo) / desc[b2.inst].n_tiles;
    return wa > wb;
  });

  cfs_batch *b = new cfs_batch();
  b->device = dev;
  b->n = n_items;
  b->plan = p;
  b->cus = cus;
  b->n_items32 = n32;
  b->n_items64 = static_cast<uint32_t>(emit.size()) - n32;
  b->n_direct32 = d32;
  b->n_direct64 = static_cast<uint32_t>(direct.size()) - d32;
  b->n_acc = static_cast<uint32_t>(acc.size());
  b->n_trans = static_cast<uint32_t>(trans.size());
  for (int i = 0; i < n_items; ++i) b->n_maps.push_back(items[i].sys.n_maps);
  HIP_TRY(hipMalloc(&b->d_desc, sizeof(InstDesc) * n_items), "hipMalloc(descriptors)");
  HIP_TRY(hipMalloc(&b->d_items, sizeof(EmitItem) * std::max<size_t>(emit.size() + direct.size(), 1)),
          "hipMalloc(items)");
  HIP_TRY(hipMalloc(&b->d_acc, sizeof(AccItem) * std::max<size_t>(acc.size(), 1)), "hipMalloc(acc)");
  HIP_TRY(hipMalloc(&b->d_queues, kQueues * sizeof(uint32_t)), "hipMalloc(queues)");
  if (!emit.empty()) {
    HIP_TRY(hipMalloc(&b->d_records, std::max<uint64_t>(rec_total, 1) * sizeof(uint16_t)),
            "hipMalloc(records)");
    HIP_TRY(hipMalloc(&b->d_tables, std::max<uint64_t>(table_total, 1) * sizeof(uint16_t)),
            "hipMalloc(tables)");
    HIP_TRY(hipMalloc(&b->d_ctables, std::max<uint64_t>(table_total, 1) * sizeof(uint16_t)),
            "hipMalloc(chunk tables)");
    HIP_TRY(hipMalloc(&b->d_trans, sizeof(TransItem) * std::max<size_t>(trans.size(), 1)),
            "hipMalloc(transpose items)");
    if (!trans.empty())
      HIP_TRY(hipMemcpy(b->d_trans, trans.data(), sizeof(TransItem) * trans.size(),
                        hipMemcpyHostToDevice),
              "copy transpose items");
  }
  HIP_TRY(hipMemcpy(b->d_desc, desc.data(), sizeof(InstDesc) * n_items, hipMemcpyHostToDevice),
          "copy descriptors");
  if (!emit.empty())
    HIP_TRY(hipMemcpy(b->d_items, emit.data(), sizeof(EmitItem) * emit.size(), hipMemcpyHostToDevice),
            "copy items");
  if (!direct.empty())
    HIP_TRY(hipMemcpy(b->d_items + emit.size(), direct.data(), sizeof(EmitItem) * direct.size(),
                      hipMemcpyHostToDevice),
            "copy direct items");
  if (!acc.empty())
    HIP_TRY(hipMemcpy(b->d_acc, acc.data(), sizeof(AccItem) * acc.size(), hipMemcpyHostToDevice),
            "copy accumulate items");
  HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
  *out = b;
  return CFS_OK;
}

extern "C" int cfs_batch_run(cfs_batch *b, void *stream) {
  clear_error();
  if (!b) return fail(CFS_E_INVALID, "batch is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  if (dev != b->device) return fail(CFS_E_INVALID, "batch was created on device %d, current is %d",
                                    b->device, dev);
  if (!b->exec) {
    BatchLaunch L{};
    L.desc = b->d_desc;
    L.n_inst = static_cast<uint32_t>(b->n);
    L.items = b->d_items;
    L.n_items32 = b->n_items32;
    L.n_items64 = b->n_items64;
    L.ditems = b->d_items + b->n_items32 + b->n_items64;
    L.n_direct32 = b->n_direct32;
    L.n_direct64 = b->n_direct64;
    L.acc = b->d_acc;
    L.n_acc = b->n_acc;
    L.queues = b->d_queues;
    L.records = b->d_records;
    L.ctables = b->d_ctables;
    L.tables = b->d_tables;
    L.trans = b->d_trans;
    L.n_trans = b->n_trans;
    L.emit_grid = static_cast<uint32_t>(b->plan.emit_grid);
    L.acc_grid = static_cast<uint32_t>(b->plan.acc_grid);
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_status(e, "hipStreamBeginCapture");
    const hipError_t le = launch_batch(L, b->capture_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &g);
    if (le != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return device_status(le, "batch kernels");
    }
    if (e != hipSuccess) return device_status(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      return device_status(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->exec = x;
  }
  return device_status(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

extern "C" int cfs_batch_update(cfs_batch *b, int32_t index, const cfs_system *sys, void *stream) {
  clear_error();
  if (!b) return fail(CFS_E_INVALID, "batch is NULL");
  if (index < 0 || index >= b->n) return fail(CFS_E_INVALID, "index %d outside 0..%d", index, b->n - 1);
  int rc = validate_system(sys);
  if (rc) return rc;
  if (sys->dim != 2 || sys->final_kind != CFS_FINAL_IDENTITY)
    return fail(CFS_E_UNSUPPORTED, "2D systems with the identity transform only");
  if (sys->kind)
    for (int m = 0; m < sys->n_maps; ++m)
      if (sys->kind[m] != CFS_MAP_AFFINE) return fail(CFS_E_UNSUPPORTED, "affine maps only");
  if (sys->n_maps != b->n_maps[index])
    return fail(CFS_E_INVALID, "instance %d has %d maps, the update has %d", index, b->n_maps[index],
                sys->n_maps);
  MapTable<2> mt;
  bool equal = false;
  rc = pack_table<2>(sys, &mt, &equal);
  if (rc) return rc;
  return device_status(launch_batch_set_table(b->d_desc, static_cast<uint32_t>(index), mt, equal,
                                              static_cast<hipStream_t>(stream)),
                       "cfs_batch_update");
}

extern "C" int cfs_batch_plan(const cfs_batch *b, cfs_plan *out) {
  clear_error();
  if (!b || !out) return fail(CFS_E_INVALID, "batch or out is NULL");
  *out = b->plan;
  return CFS_OK;
}

extern "C" void cfs_batch_destroy(cfs_batch *b) {
  if (!b) return;
  hipDeviceSynchronize();
  free_batch(b);
}

namespace {

// Signature of a batch's shapes (FNV-1a, 64 bits): what the timing of a plan
// depends on, not the map coefficients.
std::string batch_signature(const cfs_batch_item *items, int32_t n_items) {
  uint64_t h = 1469598103934665603ull;
  const auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFFu;
      h *= 1099511628211ull;
    }
  };
  mix(static_cast<uint64_t>(n_items));
  for (int i = 0; i < n_items; ++i) {
    const cfs_batch_item &it = items[i];
    mix(static_cast<uint64_t>(it.sys.n_maps));
    mix(it.sys.prob ? 1u : 0u);
    mix(it.run.n_points);
    mix(it.run.n_iters);
    mix(it.run.burn_in);
    mix(static_cast<uint64_t>(it.img.width) << 32 | static_cast<uint32_t>(it.img.height));
    mix(static_cast<uint64_t>(it.img.channels));
    mix(static_cast<uint64_t>(it.run.precision));
  }
  char buf[17];
  std::snprintf(buf, sizeof buf, "%016llx", static_cast<unsigned long long>(h));
  return buf;
}

// The last line of the cache file with this key, if any.
bool cache_lookup(const char *path, const std::string &arch, int cus, const std::string &sig,
                  cfs_plan *out) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char a[256], sg[32];
    int c = 0, bpi = 0, eg = 0, ag = 0, sp = 0;
    unsigned long long db = 0;
    const int got = std::sscanf(
        line,
        "{\"arch\": \"%255[^\"]\", \"cus\": %d, \"signature\": \"%31[0-9a-f]\", \"plan\": "
        "{\"blocks_per_item\": %d, \"emit_grid\": %d, \"acc_grid\": %d, \"splat_path\": %d, "
        "\"direct_below\": %llu}",
        a, &c, sg, &bpi, &eg, &ag, &sp, &db);
    if (got == 8 && arch == a && c == cus && sig == sg) {
      *out = cfs_plan{bpi, eg, ag, sp, static_cast<uint64_t>(db)};
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &arch, int cus, const std::string &sig,
                 const cfs_plan &p, float ms) {
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"arch\": \"%s\", \"cus\": %d, \"signature\": \"%s\", \"plan\": "
               "{\"blocks_per_item\": %d, \"emit_grid\": %d, \"acc_grid\": %d, "
               "\"splat_path\": %d, \"direct_below\": %llu}, \"ms\": %.4f}\n",
               arch.c_str(), cus, sig.c_str(), p.blocks_per_item, p.emit_grid, p.acc_grid,
               p.splat_path, static_cast<unsigned long long>(p.direct_below), ms);
  std::fclose(f);
}

// Milliseconds per graph launch of a batch built with plan c: a capture and
// three warm-up launches, then three timed launches.
int time_plan(const cfs_batch_item *items, int32_t n_items, const cfs_plan &c, void *stream,
              hipEvent_t ev0, hipEvent_t ev1, float *ms) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  cfs_batch *b = nullptr;
  int rc = cfs_batch_create(items, n_items, &c, &b);
  if (rc) return rc;
  for (int r = 0; r < 4 && !rc; ++r) rc = cfs_batch_run(b, stream);
  if (!rc) {
    hipError_t e = hipEventRecord(ev0, s);
    for (int r = 0; r < 3 && !rc; ++r) rc = cfs_batch_run(b, stream);
    if (e == hipSuccess) e = hipEventRecord(ev1, s);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev0, ev1);
    if (e != hipSuccess && !rc) rc = device_status(e, "autotune timing");
  }
  cfs_batch_destroy(b);
  return rc;
}

}  // namespace

extern "C" int cfs_autotune(const cfs_batch_item *items, int32_t n_items, cfs_plan *out,
                            const char *cache_path, void *stream) {
  clear_error();
  if (!out) return fail(CFS_E_INVALID, "out is NULL");
  if (!items || n_items < 1) return fail(CFS_E_INVALID, "need at least one batch item");
  for (int i = 0; i < n_items; ++i) {
    const int rc = validate_item(items[i], i);
    if (rc) return rc;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return device_status(e, "device query");
  const int cus = prop.multiProcessorCount;
  const std::string arch = prop.gcnArchName;
  const std::string sig = batch_signature(items, n_items);
  if (cache_path && cache_lookup(cache_path, arch, cus, sig, out)) return CFS_OK;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
    if (ev0) hipEventDestroy(ev0);
    return device_status(e, "hipEventCreate");
  }
  // shapes: work-item sizes and accumulate grids of the binned splat, and
  // the direct splat for the whole batch
  std::vector<cfs_plan> cands;
  for (int bpi : {1, 2, 4})
    for (int accm : {2, 4}) cands.push_back(cfs_plan{bpi, 2 * cus, accm * cus, CFS_SPLAT_BINNED, 0});
  for (int bpi : {1, 4}) cands.push_back(cfs_plan{bpi, 2 * cus, 0, CFS_SPLAT_DIRECT, 0});
  float best = 1e30f;
  cfs_plan best_plan{};
  int rc = CFS_OK;
  for (const cfs_plan &c : cands) {
    float ms = 0.0f;
    rc = time_plan(items, n_items, c, stream, ev0, ev1, &ms);
    if (rc) break;
    if (ms < best) {
      best = ms;
      best_plan = c;
    }
  }
  // then the per-instance strategy on the fastest binned shape: instances
  // below a splat threshold take the direct splat
  if (!rc && best_plan.splat_path == CFS_SPLAT_BINNED) {
    const cfs_plan shape = best_plan;
    for (uint64_t below : {1ull << 17, 1ull << 19, 1ull << 21}) {
      cfs_plan c = shape;
      c.direct_below = below;
      float ms = 0.0f;
      rc = time_plan(items, n_items, c, stream, ev0, ev1, &ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        best_plan = c;
      }
    }
  }
  hipEventDestroy(ev0);
  hipEventDestroy(ev1);
  if (rc) return rc;
  *out = best_plan;
  if (cache_path) cache_store(cache_path, arch, cus, sig, best_plan, best / 3.0f);
  return CFS_OK;
}
