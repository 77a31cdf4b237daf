// cfs_api.hip -- the C ABI (include/cfs.h): host-side validation, packing of
// the map table into kernel arguments, dispatch to the kernels, and error
// reporting through a thread-local message.  Every argument is checked
// before anything is enqueued, so a failed call writes nothing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>

#include "cfs.h"
#include "cfs_api_internal.hpp"
#include "cfs_host.hpp"

namespace cfs {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int device_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return CFS_OK;
  return fail(CFS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Selection thresholds (the library's own computation; the paper does not
// fix a rule): thresh[i] = ceil(2^32 P_i) for the FP64 left-to-right
// cumulative probabilities, or ceil((i+1) 2^32 / n) for equal ones; the last
// threshold is 2^32.
int make_thresholds(const double *prob, int n, uint64_t *thresh) {
  const uint64_t two32 = 1ull << 32;
  if (!prob) {
    for (int i = 0; i < n; ++i)
      thresh[i] = ((static_cast<uint64_t>(i) + 1) * two32 + static_cast<uint64_t>(n - 1)) /
                  static_cast<uint64_t>(n);
    return CFS_OK;
  }
  double cum = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(prob[i]) || prob[i] < 0.0)
      return fail(CFS_E_INVALID, "prob[%d] = %g is not a finite non-negative number", i, prob[i]);
    cum += prob[i];
    const double scaled = std::ceil(std::ldexp(cum, 32));
    thresh[i] = scaled >= std::ldexp(1.0, 32) ? two32 : static_cast<uint64_t>(scaled);
  }
  if (std::fabs(cum - 1.0) > 1e-6)
    return fail(CFS_E_INVALID, "probabilities sum to %.9g, not 1", cum);
  thresh[n - 1] = two32;
  return CFS_OK;
}

int validate_system(const cfs_system *s) {
  if (!s) return fail(CFS_E_INVALID, "system is NULL");
  if (s->dim != 2 && s->dim != 3) return fail(CFS_E_INVALID, "dim must be 2 or 3 (got %d)", s->dim);
  if (s->n_maps < 1 || s->n_maps > CFS_MAX_MAPS)
    return fail(CFS_E_INVALID, "n_maps must be in 1..%d (got %d)", CFS_MAX_MAPS, s->n_maps);
  if (!s->A || !s->b) return fail(CFS_E_INVALID, "map table A/b is NULL");
  const int d = s->dim;
  for (int i = 0; i < s->n_maps * d * d; ++i)
    if (!std::isfinite(s->A[i])) return fail(CFS_E_INVALID, "A[%d] is not finite", i);
  for (int i = 0; i < s->n_maps * d; ++i)
    if (!std::isfinite(s->b[i])) return fail(CFS_E_INVALID, "b[%d] is not finite", i);
  for (int i = 0; i < 24; ++i)
    if (!std::isfinite(s->final_params[i]))
      return fail(CFS_E_INVALID, "final_params[%d] is not finite", i);
  switch (s->final_kind) {
    case CFS_FINAL_IDENTITY: break;
    case CFS_FINAL_SWIRL:
    case CFS_FINAL_STRETCH:
    case CFS_FINAL_RING:
      if (d != 2) return fail(CFS_E_INVALID, "final kind %d needs dim 2", s->final_kind);
      break;
    case CFS_FINAL_TWIST_CAMERA:
      if (d != 3) return fail(CFS_E_INVALID, "twist/camera transform needs dim 3");
      break;
    default: return fail(CFS_E_INVALID, "unknown final kind %d", s->final_kind);
  }
  if (s->kind)
    for (int i = 0; i < s->n_maps; ++i) {
      if (s->kind[i] != CFS_MAP_AFFINE && s->kind[i] != CFS_MAP_CIRCLE)
        return fail(CFS_E_INVALID, "kind[%d] = %d is not a map kind", i, s->kind[i]);
      if (s->kind[i] == CFS_MAP_CIRCLE && d != 2)
        return fail(CFS_E_INVALID, "circle maps need dim 2");
    }
  if (s->compose != CFS_COMPOSE_COPY && s->compose != CFS_COMPOSE_REUSE)
    return fail(CFS_E_INVALID, "compose = %d is not a composition mode", s->compose);
  if (s->compose == CFS_COMPOSE_REUSE && d != 2)
    return fail(CFS_E_INVALID, "reuse composition needs a 2D transform (dim 2)");
  uint64_t th[CFS_MAX_MAPS];
  return make_thresholds(s->prob, s->n_maps, th);
}

int validate_run(const cfs_run *r) {
  if (!r) return fail(CFS_E_INVALID, "run is NULL");
  if (r->n_iters < 1 || r->n_iters > (1u << 20))
    return fail(CFS_E_INVALID, "n_iters must be in 1..2^20 (got %u)", r->n_iters);
  if (r->iter_offset % 4 != 0 || r->iter_offset > (1u << 30))
    return fail(CFS_E_INVALID, "iter_offset must be a multiple of 4 in 0..2^30 (got %u)",
                r->iter_offset);
  if (static_cast<uint64_t>(r->point_offset) + r->n_points > (1ull << 32))
    return fail(CFS_E_INVALID, "point_offset + n_points exceeds 2^32");
  if (r->precision != CFS_PREC_F32 && r->precision != CFS_PREC_F64)
    return fail(CFS_E_INVALID, "precision must be CFS_PREC_F32 or CFS_PREC_F64");
  return CFS_OK;
}

int validate_window(const cfs_image *img) {
  if (!img) return fail(CFS_E_INVALID, "image is NULL");
  if (img->width < 1 || img->width > 65536 || img->height < 1 || img->height > 65536)
    return fail(CFS_E_INVALID, "image size %dx%d outside 1..65536", img->width, img->height);
  if (img->channels < 1) return fail(CFS_E_INVALID, "channels must be >= 1");
  const uint64_t total = static_cast<uint64_t>(img->width) * img->height * img->channels;
  if (total > (1ull << 31)) return fail(CFS_E_INVALID, "image holds more than 2^31 elements");
  for (int a = 0; a < 2; ++a) {
    if (!std::isfinite(img->lo[a]) || !std::isfinite(img->hi[a]) || !(img->hi[a] > img->lo[a]))
      return fail(CFS_E_INVALID, "window axis %d needs finite lo < hi", a);
  }
  if (!img->data) return fail(CFS_E_INVALID, "image data is NULL");
  const size_t align = img->kind == CFS_IMAGE_U64_DEPTH ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(img->data) % align)
    return fail(CFS_E_INVALID, "image data is not %zu-byte aligned", align);
  if (img->kind == CFS_IMAGE_U64_DEPTH) {
    if (!img->density) return fail(CFS_E_INVALID, "depth image needs a density buffer");
    if (reinterpret_cast<uintptr_t>(img->density) % 4)
      return fail(CFS_E_INVALID, "density is not 4-byte aligned");
    if (img->channels != 1) return fail(CFS_E_INVALID, "depth image has one channel");
  }
  if (img->dropped && reinterpret_cast<uintptr_t>(img->dropped) % 8)
    return fail(CFS_E_INVALID, "dropped counter is not 8-byte aligned");
  return CFS_OK;
}

Window make_window(const cfs_image *img, bool by_index) {
  Window w{};
  w.width = img->width;
  w.height = img->height;
  w.channels = img->channels;
  w.by_index = by_index ? 1 : 0;
  for (int a = 0; a < 2; ++a) {
    w.lo[a] = static_cast<double>(img->lo[a]);
    const double extent = static_cast<double>(img->hi[a]) - static_cast<double>(img->lo[a]);
    w.scale[a] = static_cast<double>(a == 0 ? img->width : img->height) / extent;
  }
  return w;
}

int validate_fresh_run(const cfs_run *r) {
  const int rc = validate_run(r);
  if (rc) return rc;
  if (r->iter_offset)
    return fail(CFS_E_UNSUPPORTED, "continued runs (iter_offset %u) are for cfs_chaos_game only",
                r->iter_offset);
  if (r->burn_in > r->n_iters)
    return fail(CFS_E_INVALID, "burn_in %u exceeds n_iters %u", r->burn_in, r->n_iters);
  return CFS_OK;
}

cfs_run call_run(const cfs_run *r) {
  cfs_run c = *r;
  const uint32_t b = r->burn_in > r->iter_offset ? r->burn_in - r->iter_offset : 0u;
  c.burn_in = b < r->n_iters ? b : r->n_iters;
  return c;
}

RunArgs make_run_args(const cfs_run *r) {
  RunArgs ra{};
  ra.k0 = static_cast<uint32_t>(r->seed);
  ra.k1 = static_cast<uint32_t>(r->seed >> 32);
  ra.instance = r->instance;
  ra.n_points = r->n_points;
  ra.point_offset = r->point_offset;
  ra.n_iters = r->n_iters;
  ra.burn_in = r->burn_in;
  ra.iter_block = r->iter_offset / 4;
  return ra;
}

template <int DIM>
int pack_table(const cfs_system *s, MapTable<DIM> *mt, bool *equal) {
  std::memset(mt, 0, sizeof *mt);
  const int n = s->n_maps;
  constexpr int C = DIM * (DIM + 1);
  for (int m = 0; m < n; ++m) {
    for (int r = 0; r < DIM; ++r) {
      for (int c = 0; c < DIM; ++c) mt->coef[m * C + r * DIM + c] = s->A[(m * DIM + r) * DIM + c];
      mt->coef[m * C + DIM * DIM + r] = s->b[m * DIM + r];
    }
  }
  mt->n_maps = n;
  mt->flags = 0;
  mt->circle_mask = 0;
  if (s->kind)
    for (int m = 0; m < n; ++m)
      if (s->kind[m] == CFS_MAP_CIRCLE) {
        mt->circle_mask |= 1ull << m;
        mt->flags |= kFlagCircle;
      }
  if (s->compose == CFS_COMPOSE_REUSE) mt->flags |= kFlagReuse;
  // one linear part for every map (compared bit for bit): the kernels then
  // gather only the translations; a multiple of the identity (and no
  // negative-zero translation) takes one FMA per coordinate
  mt->lin = mt->flags & kFlagCircle ? kLinGeneral : kLinShared;
  for (int m = 1; m < n && mt->lin != kLinGeneral; ++m)
    if (std::memcmp(&mt->coef[m * C], &mt->coef[0], sizeof(float) * DIM * DIM) != 0)
      mt->lin = kLinGeneral;
  if (mt->lin == kLinShared) {
    bool scalar = true;
    for (int r = 0; r < DIM; ++r)
      for (int c = 0; c < DIM; ++c)
        scalar = scalar && (r == c ? mt->coef[r * DIM + c] == mt->coef[0] : mt->coef[r * DIM + c] == 0.0f);
    for (int i = 0; i < n * DIM; ++i) scalar = scalar && !(s->b[i] == 0.0f && std::signbit(s->b[i]));
    if (scalar) mt->lin = kLinScalar;
  }
  uint64_t th[CFS_MAX_MAPS];
  const int rc = make_thresholds(s->prob, n, th);
  if (rc) return rc;
  *equal = (s->prob == nullptr);
  if (*equal) {
    mt->n_search = 0;
    return CFS_OK;
  }
  // maps past the first threshold that reaches 2^32 can never be drawn
  int ns = n;
  for (int i = 0; i < n; ++i)
    if (th[i] >= (1ull << 32)) {
      ns = i + 1;
      break;
    }
  for (int i = 0; i < ns - 1; ++i) mt->thresh[i] = static_cast<uint32_t>(th[i]);
  mt->n_search = ns;
  return CFS_OK;
}

template int pack_table<2>(const cfs_system *, MapTable<2> *, bool *);
template int pack_table<3>(const cfs_system *, MapTable<3> *, bool *);

}  // namespace cfs

using namespace cfs;

extern "C" int cfs_version(void) { return CFS_VERSION; }

extern "C" const char *cfs_last_error(void) { return g_last_error.c_str(); }

extern "C" int cfs_image_clear(const cfs_image *img, void *stream) {
  clear_error();
  int rc = validate_window(img);
  if (rc) return rc;
  const size_t n = static_cast<size_t>(img->width) * img->height * img->channels;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  switch (img->kind) {
    case CFS_IMAGE_U32_COUNT:
    case CFS_IMAGE_F32_DENSITY:  // +0.0f has the all-zero bit pattern
      e = launch_clear_u32(static_cast<uint32_t *>(img->data), n, s);
      break;
    case CFS_IMAGE_U64_DEPTH:
      e = launch_fill_u64(static_cast<unsigned long long *>(img->data), n, ~0ull, s);
      if (e == hipSuccess) e = launch_clear_u32(img->density, n, s);
      break;
    default: return fail(CFS_E_INVALID, "unknown image kind %d", img->kind);
  }
  if (e == hipSuccess && img->dropped) e = launch_fill_u64(img->dropped, 1, 0ull, s);
  return device_status(e, "cfs_image_clear");
}

namespace {

// Records of one launch of the binned path: 2^29 16-bit count records
// (1 GiB) or 2^30 8-byte depth records (8 GiB), which keeps record indices
// within 31 bits and chunk indices within 24 (the kernels index records in
// 32-bit arithmetic).  Each launch ends with a read-modify-write of the
// image's occupied tiles and each accumulate workgroup's tail, so depth runs
// (192 MiB of image) take the larger budget: the 3D workload of 2^26 points
// x 16 splats is one launch (four launches of 2^28 records took 2.5% longer).
uint64_t binned_record_budget(bool depth) { return depth ? (1ull << 30) : (1ull << 29); }

uint64_t binned_block_records(const cfs_run *run, bool depth, uint32_t per_iter) {
  const uint64_t slots = depth ? kDSlots : kBinSlots;
  const uint64_t cap = depth ? kDCap : kChunkCap;
  const uint64_t flushes =
      (static_cast<uint64_t>(run->n_iters - run->burn_in) * per_iter + slots - 1) / slots;
  return flushes * cap;
}

// Whether one workgroup's records fit the budget of a launch (runs of more
// than about 10^6 splats per point do not, and take the direct splat).
bool binned_fits(const cfs_run *run, bool depth, uint32_t per_iter = 1) {
  return binned_block_records(run, depth, per_iter) <= binned_record_budget(depth);
}

// Points per launch of the binned path: few enough that the records of one
// launch stay within binned_record_budget() (the caller has checked
// binned_fits(), so one workgroup's records always do), and for count images
// at most 2^24.
uint32_t binned_slice(const cfs_run *run, bool depth, uint32_t per_iter = 1) {
  uint64_t max_blocks = binned_record_budget(depth) / binned_block_records(run, depth, per_iter);
  if (max_blocks < 1) max_blocks = 1;
  uint64_t pts = max_blocks * (depth ? kDBlock : kBinBlock);
  if (!depth && pts > (1ull << 24)) pts = 1ull << 24;
  if (pts > run->n_points) pts = run->n_points;
  return static_cast<uint32_t>(pts);
}

// Whether this call takes the binned splat (arguments already validated).
bool use_binned(const cfs_run *run, const cfs_image *img) {
  if (run->splat_path == CFS_SPLAT_DIRECT) return false;
  if (img->kind != CFS_IMAGE_U32_COUNT && img->kind != CFS_IMAGE_U64_DEPTH) return false;
  if (run->n_iters == run->burn_in || run->n_points == 0) return false;
  const uint64_t elems = static_cast<uint64_t>(img->width) * img->height * img->channels;
  const bool depth = img->kind == CFS_IMAGE_U64_DEPTH;
  const uint64_t tile = depth ? kDTileElems : kTileElems;
  if (elems > static_cast<uint64_t>(kMaxTiles) * tile) return false;
  if (!binned_fits(run, depth)) return false;
  if (run->splat_path == CFS_SPLAT_BINNED) return true;
  return static_cast<uint64_t>(run->n_points) * (run->n_iters - run->burn_in) >= (1ull << 20);
}

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Workspace of one launch of `points` points: records, the run table and its
// transpose, and the transpose's column sums.
size_t binned_workspace_for(uint32_t points, const cfs_run *run, const cfs_image *img,
                            uint32_t per_iter = 1) {
  const uint32_t elems = static_cast<uint32_t>(img->width) * img->height * img->channels;
  const bool depth = img->kind == CFS_IMAGE_U64_DEPTH;
  const BinPlan bp = bin_plan(points, run->n_iters, run->burn_in, elems, depth, per_iter);
  return align_up(bp.records_bytes) + 2 * align_up(bp.table_bytes) + align_up(bp.sums_bytes);
}

size_t binned_workspace(const cfs_run *run, const cfs_image *img, uint32_t per_iter = 1) {
  const bool depth = img->kind == CFS_IMAGE_U64_DEPTH;
  return binned_workspace_for(binned_slice(run, depth, per_iter), run, img, per_iter);
}

// Points per launch of the binned path whose workspace takes at most `bytes`:
// the most whole workgroups of points (at most binned_slice()) that fit, or 0
// when one workgroup's records and tables alone do not.  The workspace grows
// with the points of a launch, so a bisection over workgroups finds it.
uint32_t binned_slice_within(const cfs_run *run, const cfs_image *img, size_t bytes) {
  const bool depth = img->kind == CFS_IMAGE_U64_DEPTH;
  const uint32_t top = binned_slice(run, depth);
  const uint32_t block = depth ? kDBlock : kBinBlock;
  const auto pts_of = [&](uint32_t blocks) { return std::min<uint32_t>(top, blocks * block); };
  uint32_t lo = 0, hi = (top + block - 1) / block;  // fits(lo) holds, answer <= hi
  if (binned_workspace_for(pts_of(1), run, img) > bytes) return 0;
  lo = 1;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1) / 2;
    if (binned_workspace_for(pts_of(mid), run, img) <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return pts_of(lo);
}

// Point the binned arguments of one slice into the workspace.
void bind_workspace(BinArgs *ba, const BinPlan &bp, void *workspace) {
  ba->records = static_cast<uint16_t *>(workspace);
  ba->drecords = static_cast<uint2 *>(workspace);
  char *tables = static_cast<char *>(workspace) + align_up(bp.records_bytes);
  ba->chunk_start = reinterpret_cast<uint16_t *>(tables);
  ba->tile_start = reinterpret_cast<uint16_t *>(tables + align_up(bp.table_bytes));
  ba->tile_sums = bp.sums_bytes
                      ? reinterpret_cast<uint32_t *>(tables + 2 * align_up(bp.table_bytes))
                      : nullptr;
  ba->n_rb = bp.n_rb;
  ba->n_chunks = bp.n_chunks;
  ba->flushes = bp.flushes;
  ba->n_tiles = bp.n_tiles;
  ba->elems = bp.elems;
  ba->parts = bp.parts;
  ba->log2g = bp.log2g;
}

// Scene objects: validation and packing into kernel arguments.
int validate_objects(const cfs_object *objects, int32_t n_objects, const cfs_image *img) {
  if (!objects) return fail(CFS_E_INVALID, "objects is NULL");
  if (n_objects < 1 || n_objects > CFS_MAX_OBJECTS)
    return fail(CFS_E_INVALID, "n_objects must be in [1, %d] (got %d)", CFS_MAX_OBJECTS,
                n_objects);
  for (int o = 0; o < n_objects; ++o) {
    const cfs_object &ob = objects[o];
    if (ob.final_kind != CFS_FINAL_IDENTITY && ob.final_kind != CFS_FINAL_SWIRL &&
        ob.final_kind != CFS_FINAL_STRETCH && ob.final_kind != CFS_FINAL_RING)
      return fail(CFS_E_INVALID, "object %d: final_kind %d is not a 2D transform", o,
                  ob.final_kind);
    for (int i = 0; i < 24; ++i)
      if (!std::isfinite(ob.final_params[i]))
        return fail(CFS_E_INVALID, "object %d: final_params[%d] is not finite", o, i);
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(ob.place[i]))
        return fail(CFS_E_INVALID, "object %d: place[%d] is not finite", o, i);
    if (!std::isfinite(ob.copy_lo[0]) || !std::isfinite(ob.copy_lo[1]) ||
        !std::isfinite(ob.copy_span[0]) || !std::isfinite(ob.copy_span[1]) ||
        !std::isfinite(ob.scale_lo) || !std::isfinite(ob.scale_span))
      return fail(CFS_E_INVALID, "object %d: copy placement is not finite", o);
    if (ob.channel < 0 || ob.channel >= img->channels)
      return fail(CFS_E_INVALID, "object %d: channel %d outside [0, %d)", o, ob.channel,
                  img->channels);
    if (ob.n_copies < 1 || ob.n_copies > (1u << 24))
      return fail(CFS_E_INVALID, "object %d: n_copies must be in [1, 2^24]", o);
  }
  return CFS_OK;
}

SceneArgs pack_objects(const cfs_object *objects, int32_t n_objects) {
  SceneArgs sc;
  std::memset(&sc, 0, sizeof sc);
  sc.n_obj = n_objects;
  uint32_t rows = 0;  // LDS placement rows handed out so far
  for (int o = 0; o < n_objects; ++o) {
    const cfs_object &ob = objects[o];
    SceneObject &d = sc.obj[o];
    d.kind = ob.final_kind;
    d.channel = ob.channel;
    d.n_copies = ob.n_copies;
    std::memcpy(d.fp, ob.final_params, sizeof d.fp);
    std::memcpy(d.place, ob.place, sizeof d.place);
    d.copy_lo[0] = ob.copy_lo[0];
    d.copy_lo[1] = ob.copy_lo[1];
    d.copy_span[0] = ob.copy_span[0];
    d.copy_span[1] = ob.copy_span[1];
    d.scale_lo = ob.scale_lo;
    d.scale_span = ob.scale_span;
    d.tab_base = -1;
    if (ob.n_copies > 1) {
      sc.any_copies = 1;
      if (ob.n_copies <= kSceneCopyTable - rows) {
        d.tab_base = static_cast<int32_t>(rows);
        rows += ob.n_copies;
      }
    }
  }
  return sc;
}

int validate_scene(const cfs_system *sys, const cfs_object *objects, int32_t n_objects,
                   const cfs_run *run, const cfs_image *img) {
  int rc = validate_system(sys);
  if (!rc) rc = validate_fresh_run(run);
  if (!rc) rc = validate_window(img);
  if (rc) return rc;
  if (sys->dim != 2) return fail(CFS_E_INVALID, "a scene's primitive must be 2D");
  if (sys->final_kind != CFS_FINAL_IDENTITY || sys->compose != CFS_COMPOSE_COPY)
    return fail(CFS_E_INVALID,
                "a scene's primitive has no transform of its own (the objects carry them)");
  if (img->kind != CFS_IMAGE_U32_COUNT)
    return fail(CFS_E_INVALID, "cfs_chaos_scene renders U32_COUNT images");
  if (run->splat_path < CFS_SPLAT_AUTO || run->splat_path > CFS_SPLAT_BINNED)
    return fail(CFS_E_INVALID, "unknown splat_path %d", run->splat_path);
  return validate_objects(objects, n_objects, img);
}

bool scene_binned(const cfs_run *run, const cfs_image *img, int32_t n_objects) {
  if (run->splat_path == CFS_SPLAT_DIRECT) return false;
  if (run->n_iters == run->burn_in || run->n_points == 0) return false;
  const uint64_t elems = static_cast<uint64_t>(img->width) * img->height * img->channels;
  if (elems > static_cast<uint64_t>(kMaxTiles) * kTileElems) return false;
  if (!binned_fits(run, false, static_cast<uint32_t>(n_objects))) return false;
  if (run->splat_path == CFS_SPLAT_BINNED) return true;
  return static_cast<uint64_t>(run->n_points) * (run->n_iters - run->burn_in) * n_objects >=
         (1ull << 20);
}

}  // namespace

extern "C" size_t cfs_chaos_game_workspace(const cfs_system *sys, const cfs_run *run,
                                           const cfs_image *img) {
  if (validate_system(sys) || validate_run(run) || validate_window(img)) return 0;
  const cfs_run cr = call_run(run);
  if (!use_binned(&cr, img)) return 0;
  return binned_workspace(&cr, img);
}

namespace cfs {

// Validation, packing and the launch plan of one cfs_chaos_game call.  With
// `budget` > 0 the binned path cuts the run into launches whose workspace
// takes at most `budget` bytes (a run that cannot be cut that fine takes the
// direct splat under CFS_SPLAT_AUTO and is refused under CFS_SPLAT_BINNED).
int chaos_prepare(const cfs_system *sys, const cfs_run *run_in, const cfs_image *img,
                  void *final_points, uint8_t *last_index, uint8_t *indices, size_t budget,
                  ChaosCall *call_out) {
  int rc = validate_system(sys);
  if (!rc) rc = validate_run(run_in);
  if (!rc) rc = validate_window(img);
  if (rc) return rc;
  if (run_in->iter_offset && !final_points)
    return fail(CFS_E_INVALID, "a continued run (iter_offset %u) reads its start from final_points",
                run_in->iter_offset);
  // this call's view of the run: the part of the burn-in inside it
  ChaosCall &cc = *call_out;
  std::memset(&cc, 0, sizeof cc);
  cc.run = call_run(run_in);
  const cfs_run *run = &cc.run;
  if (run->splat_path < CFS_SPLAT_AUTO || run->splat_path > CFS_SPLAT_BINNED)
    return fail(CFS_E_INVALID, "unknown splat_path %d", run->splat_path);
  ChaosJob &job = cc.job;
  job.dim = sys->dim;
  job.final_kind = sys->final_kind;
  job.precision = run->precision;
  if (img->kind == CFS_IMAGE_U32_COUNT) {
    if (sys->final_kind == CFS_FINAL_TWIST_CAMERA)
      return fail(CFS_E_UNSUPPORTED, "the camera transform renders into a U64 depth image");
    if (img->channels != 1 && img->channels != sys->n_maps)
      return fail(CFS_E_INVALID, "channels must be 1 or n_maps (%d), got %d", sys->n_maps,
                  img->channels);
    job.depth = false;
  } else if (img->kind == CFS_IMAGE_U64_DEPTH) {
    if (sys->final_kind != CFS_FINAL_TWIST_CAMERA)
      return fail(CFS_E_UNSUPPORTED, "a depth image needs the twist/camera transform");
    // keys order splats by the FP32 bit pattern of their depth, which is
    // the order of the depths only for non-negative values
    if (!std::isfinite(img->near_plane) || !(img->near_plane >= 0.0f))
      return fail(CFS_E_INVALID, "near_plane must be finite and >= 0 (got %g)",
                  static_cast<double>(img->near_plane));
    job.depth = true;
  } else {
    return fail(CFS_E_INVALID, "cfs_chaos_game renders U32_COUNT or U64_DEPTH images");
  }
  const uint64_t elems = static_cast<uint64_t>(img->width) * img->height * img->channels;
  const uint64_t tile = job.depth ? kDTileElems : kTileElems;
  if (run->splat_path == CFS_SPLAT_BINNED && elems > static_cast<uint64_t>(kMaxTiles) * tile)
    return fail(CFS_E_UNSUPPORTED, "binned splat handles images of at most %u elements",
                static_cast<unsigned>(kMaxTiles * tile));
  if (run->splat_path == CFS_SPLAT_BINNED && run->n_iters > run->burn_in &&
      !binned_fits(run, job.depth))
    return fail(CFS_E_UNSUPPORTED,
                "binned splat: %u splatted steps per point exceed one launch's record budget",
                run->n_iters - run->burn_in);
  const size_t align = run->precision == CFS_PREC_F64 ? 8 : 4;
  if (final_points && reinterpret_cast<uintptr_t>(final_points) % align)
    return fail(CFS_E_INVALID, "final_points is not %zu-byte aligned", align);
  job.binned = use_binned(run, img);
  if (job.binned) {
    cc.slice = budget ? binned_slice_within(run, img, budget) : binned_slice(run, job.depth);
    if (cc.slice == 0) {
      if (run->splat_path == CFS_SPLAT_BINNED)
        return fail(CFS_E_UNSUPPORTED,
                    "binned splat: one workgroup's records (%u splatted steps per point) "
                    "exceed the %zu-byte workspace limit",
                    run->n_iters - run->burn_in, budget);
      job.binned = false;  // AUTO: the direct splat needs no workspace
    } else {
      cc.need = binned_workspace_for(cc.slice, run, img);
    }
  }
  if (sys->dim == 2)
    rc = pack_table<2>(sys, &job.mt2, &job.equal);
  else
    rc = pack_table<3>(sys, &job.mt3, &job.equal);
  if (rc) return rc;
  job.win = make_window(img, img->kind == CFS_IMAGE_U32_COUNT && img->channels > 1);
  job.ra = make_run_args(run);
  std::memcpy(job.fa.p, sys->final_params, sizeof job.fa.p);
  job.img = img->data;
  job.density = img->density;
  job.near_plane = img->near_plane;
  job.out.final_points = final_points;
  job.out.last_index = last_index;
  job.out.indices = indices;
  job.out.dropped = img->dropped;
  cc.elems = static_cast<uint32_t>(elems);
  return CFS_OK;
}

// Enqueue a prepared call: the direct kernel, or the binned launches of at
// most cc.slice points each, one after the other on the stream, all sharing
// `workspace` (cc.need bytes, checked by the caller).  `timed`: record the
// measurement hook's phase events.
int chaos_launch(const ChaosCall &cc, void *workspace, bool timed, hipStream_t s) {
  const ChaosJob &job = cc.job;
  const cfs_run *run = &cc.run;
  if (!job.binned) {
    ChaosJob dj = job;
    dj.ev = timed ? timing_slice() : nullptr;
    return device_status(launch_chaos(dj, s), "cfs_chaos_game");
  }
  const size_t real_bytes = run->precision == CFS_PREC_F64 ? sizeof(double) : sizeof(float);
  for (uint32_t done = 0; done < run->n_points; done += cc.slice) {
    const uint32_t pts = std::min(cc.slice, run->n_points - done);
    const BinPlan bp = bin_plan(pts, run->n_iters, run->burn_in, cc.elems, job.depth);
    ChaosJob sj = job;
    sj.ra.n_points = pts;
    sj.ra.point_offset = run->point_offset + done;
    if (job.out.final_points)
      sj.out.final_points = static_cast<char *>(job.out.final_points) +
                            static_cast<size_t>(done) * job.dim * real_bytes;
    if (job.out.last_index) sj.out.last_index = job.out.last_index + done;
    if (job.out.indices) sj.out.indices = job.out.indices + static_cast<size_t>(done) * run->n_iters;
    bind_workspace(&sj.ba, bp, workspace);
    sj.ev = timed ? timing_slice() : nullptr;
    const int rc = device_status(launch_chaos_binned(sj, s), "cfs_chaos_game");
    if (rc) return rc;
  }
  return CFS_OK;
}

}  // namespace cfs

extern "C" int cfs_chaos_game(const cfs_system *sys, const cfs_run *run_in, const cfs_image *img,
                              void *final_points, uint8_t *last_index, uint8_t *indices,
                              void *workspace, size_t workspace_bytes, void *stream) {
  clear_error();
  ChaosCall cc;
  int rc = chaos_prepare(sys, run_in, img, final_points, last_index, indices, 0, &cc);
  if (rc) return rc;
  // a workspace smaller than the fewest launches need: launches that fit it
  if (cc.job.binned && workspace && workspace_bytes < cc.need) {
    rc = chaos_prepare(sys, run_in, img, final_points, last_index, indices, workspace_bytes, &cc);
    if (rc == CFS_E_UNSUPPORTED && run_in->splat_path == CFS_SPLAT_BINNED)
      return fail(CFS_E_WORKSPACE, "binned splat: one workgroup's records exceed the %zu-byte "
                  "workspace", workspace_bytes);
    if (rc) return rc;
  }
  if (cc.job.binned) {
    if (!workspace || workspace_bytes < cc.need)
      return fail(CFS_E_WORKSPACE, "binned splat needs %zu bytes of workspace, got %zu", cc.need,
                  workspace ? workspace_bytes : static_cast<size_t>(0));
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
      return fail(CFS_E_WORKSPACE, "workspace must be 256-byte aligned");
  }
  return chaos_launch(cc, workspace, timing_begin_call(), static_cast<hipStream_t>(stream));
}

extern "C" size_t cfs_chaos_scene_workspace(const cfs_system *sys, const cfs_object *objects,
                                            int32_t n_objects, const cfs_run *run,
                                            const cfs_image *img) {
  if (validate_scene(sys, objects, n_objects, run, img)) return 0;
  if (!scene_binned(run, img, n_objects)) return 0;
  return binned_workspace(run, img, static_cast<uint32_t>(n_objects));
}

extern "C" int cfs_chaos_scene(const cfs_system *sys, const cfs_object *objects,
                               int32_t n_objects, const cfs_run *run, const cfs_image *img,
                               void *workspace, size_t workspace_bytes, void *stream) {
  clear_error();
  int rc = validate_scene(sys, objects, n_objects, run, img);
  if (rc) return rc;
  const uint64_t elems = static_cast<uint64_t>(img->width) * img->height * img->channels;
  if (run->splat_path == CFS_SPLAT_BINNED && elems > static_cast<uint64_t>(kMaxTiles) * kTileElems)
    return fail(CFS_E_UNSUPPORTED, "binned splat handles images of at most %u elements",
                static_cast<unsigned>(kMaxTiles * kTileElems));
  if (run->splat_path == CFS_SPLAT_BINNED && run->n_iters > run->burn_in &&
      !binned_fits(run, false, static_cast<uint32_t>(n_objects)))
    return fail(CFS_E_UNSUPPORTED,
                "binned splat: %u splatted steps x %d objects per point exceed one launch's "
                "record budget", run->n_iters - run->burn_in, n_objects);
  SceneJob job;
  std::memset(&job, 0, sizeof job);
  job.precision = run->precision;
  job.binned = scene_binned(run, img, n_objects);
  const uint32_t per_iter = static_cast<uint32_t>(n_objects);
  if (job.binned) {
    const size_t need = binned_workspace(run, img, per_iter);
    if (!workspace || workspace_bytes < need)
      return fail(CFS_E_WORKSPACE, "binned splat needs %zu bytes of workspace, got %zu", need,
                  workspace ? workspace_bytes : static_cast<size_t>(0));
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
      return fail(CFS_E_WORKSPACE, "workspace must be 256-byte aligned");
  }
  rc = pack_table<2>(sys, &job.mt, &job.equal);
  if (rc) return rc;
  job.win = make_window(img, false);
  job.ra = make_run_args(run);
  job.sc = pack_objects(objects, n_objects);
  job.img = static_cast<uint32_t *>(img->data);
  job.dropped = img->dropped;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!job.binned) return device_status(launch_scene(job, s), "cfs_chaos_scene");
  const uint32_t slice = binned_slice(run, false, per_iter);
  for (uint32_t done = 0; done < run->n_points; done += slice) {
    const uint32_t pts = std::min(slice, run->n_points - done);
    const BinPlan bp = bin_plan(pts, run->n_iters, run->burn_in, static_cast<uint32_t>(elems),
                                false, per_iter);
    SceneJob sj = job;
    sj.ra.n_points = pts;
    sj.ra.point_offset = run->point_offset + done;
    bind_workspace(&sj.ba, bp, workspace);
    rc = device_status(launch_scene(sj, s), "cfs_chaos_scene");
    if (rc) return rc;
  }
  return CFS_OK;
}

extern "C" int cfs_philox_dump(uint64_t seed, const uint32_t *ctrs, uint32_t *out, uint64_t n,
                               void *stream) {
  clear_error();
  if (n && (!ctrs || !out)) return fail(CFS_E_INVALID, "ctrs/out is NULL");
  if (n > (1ull << 32)) return fail(CFS_E_INVALID, "n exceeds 2^32");
  if ((reinterpret_cast<uintptr_t>(ctrs) | reinterpret_cast<uintptr_t>(out)) % 16)
    return fail(CFS_E_INVALID, "ctrs/out must be 16-byte aligned");
  return device_status(launch_philox_dump(static_cast<uint32_t>(seed),
                                          static_cast<uint32_t>(seed >> 32), ctrs, out, n,
                                          static_cast<hipStream_t>(stream)),
                       "cfs_philox_dump");
}
