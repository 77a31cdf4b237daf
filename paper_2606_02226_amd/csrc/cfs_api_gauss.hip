// cfs_api_gauss.hip -- C ABI of the differentiable form (cfs_splat,
// cfs_splat_backward and their workspace queries): validation, packing and
// point-range slicing of the Gaussian splat.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cfs.h"
#include "cfs_api_internal.hpp"
#include "cfs_host.hpp"

using namespace cfs;

namespace {

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

int validate_gauss(const cfs_system *sys, const cfs_run *run, const cfs_image *img, float sigma) {
  int rc = validate_system(sys);
  if (!rc) rc = validate_fresh_run(run);
  if (!rc) rc = validate_window(img);
  if (rc) return rc;
  if (sys->dim != 2 || sys->final_kind != CFS_FINAL_IDENTITY)
    return fail(CFS_E_UNSUPPORTED, "the Gaussian splat takes 2D systems with the identity transform");
  if (sys->kind)
    for (int i = 0; i < sys->n_maps; ++i)
      if (sys->kind[i] != CFS_MAP_AFFINE)
        return fail(CFS_E_UNSUPPORTED, "the Gaussian splat and its adjoint take affine maps only");
  if (run->precision != CFS_PREC_F32)
    return fail(CFS_E_UNSUPPORTED, "the Gaussian splat computes positions in FP32");
  if (img->kind != CFS_IMAGE_F32_DENSITY || img->channels != 1)
    return fail(CFS_E_INVALID, "the Gaussian splat renders a one-channel F32_DENSITY image");
  if (!(sigma > 0.0f) || sigma > 2.5f) return fail(CFS_E_INVALID, "sigma_px must be in (0, 2.5]");
  const uint64_t tiles = static_cast<uint64_t>((img->width + kGTile - 1) / kGTile) *
                         ((img->height + kGTile - 1) / kGTile);
  if (tiles > static_cast<uint64_t>(kGMaxTiles))
    return fail(CFS_E_UNSUPPORTED, "the Gaussian splat handles at most %d tiles of %dx%d pixels",
                kGMaxTiles, kGTile, kGTile);
  return CFS_OK;
}

// Points per forward launch: at most 2^27 records (1 GiB) of workspace.
uint32_t gauss_slice(const cfs_run *run) {
  const uint64_t flushes = std::max<uint64_t>((run->n_iters - run->burn_in + kGSlots - 1) / kGSlots, 1);
  uint64_t blocks = (1ull << 27) / (flushes * kGCap);
  if (blocks < 1) blocks = 1;
  uint64_t pts = blocks * kGBlock;
  if (pts > run->n_points) pts = run->n_points;
  return static_cast<uint32_t>(std::max<uint64_t>(pts, 1));
}

GaussParams make_gauss_params(const cfs_run *run, const cfs_image *img, float sigma) {
  GaussParams gp{};
  gp.sigma = sigma;
  gp.R = 3.0f * sigma;
  gp.inv2s2 = 1.0f / (2.0f * sigma * sigma);
  gp.inv_s2 = 1.0f / (sigma * sigma);
  gp.cutoff = std::exp(-gp.R * gp.R * gp.inv2s2);
  gp.taps = static_cast<int32_t>(std::ceil(2.0f * gp.R));
  gp.weight = static_cast<float>(1.0 / (static_cast<double>(run->n_points) *
                                        static_cast<double>(run->n_iters - run->burn_in)));
  gp.width = img->width;
  gp.height = img->height;
  gp.tiles_x = (img->width + kGTile - 1) / kGTile;
  gp.tiles_y = (img->height + kGTile - 1) / kGTile;
  for (int a = 0; a < 2; ++a) {
    gp.lo[a] = img->lo[a];
    gp.scale[a] = static_cast<float>(static_cast<double>(a == 0 ? img->width : img->height) /
                                     (static_cast<double>(img->hi[a]) - static_cast<double>(img->lo[a])));
  }
  return gp;
}

}  // namespace

extern "C" size_t cfs_splat_workspace(const cfs_system *sys, const cfs_run *run,
                                      const cfs_image *img, float sigma_px) {
  if (validate_gauss(sys, run, img, sigma_px)) return 0;
  if (run->n_iters == run->burn_in || run->n_points == 0) return 0;
  const GaussPlan p = gauss_plan(gauss_slice(run), run->n_iters, run->burn_in, img->width, img->height);
  return align_up(p.records_bytes) + 2 * align_up(p.table_bytes) + align_up(p.sums_bytes);
}

extern "C" int cfs_splat(const cfs_system *sys, const cfs_run *run, const cfs_image *img,
                         float sigma_px, float *ckpt, int32_t ckpt_every, void *workspace,
                         size_t workspace_bytes, void *stream) {
  clear_error();
  int rc = validate_gauss(sys, run, img, sigma_px);
  if (rc) return rc;
  if (ckpt && (ckpt_every < 1 || ckpt_every > kMaxSeg))
    return fail(CFS_E_INVALID, "ckpt_every must be in 1..%d", kMaxSeg);
  if (ckpt && reinterpret_cast<uintptr_t>(ckpt) % 8) return fail(CFS_E_INVALID, "ckpt is not 8-byte aligned");
  const size_t need = cfs_splat_workspace(sys, run, img, sigma_px);
  if (need && (!workspace || workspace_bytes < need))
    return fail(CFS_E_WORKSPACE, "cfs_splat needs %zu bytes of workspace, got %zu", need,
                workspace ? workspace_bytes : static_cast<size_t>(0));
  if (workspace && reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(CFS_E_WORKSPACE, "workspace must be 256-byte aligned");
  GaussJob job;
  std::memset(&job, 0, sizeof job);
  rc = pack_table<2>(sys, &job.mt, &job.equal);
  if (rc) return rc;
  job.gp = make_gauss_params(run, img, sigma_px);
  job.dens = static_cast<float *>(img->data);
  job.dropped = img->dropped;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RunArgs ra = make_run_args(run);
  const bool no_splats = run->n_iters == run->burn_in;
  const uint32_t slice = gauss_slice(run);
  for (uint32_t done = 0; done < run->n_points; done += slice) {
    const uint32_t pts = std::min(slice, run->n_points - done);
    GaussJob j = job;
    j.ra = ra;
    j.ra.n_points = pts;
    j.ra.point_offset = run->point_offset + done;
    const GaussPlan p = gauss_plan(pts, run->n_iters, run->burn_in, img->width, img->height);
    j.gb.records = static_cast<float2 *>(workspace);
    char *tables = static_cast<char *>(workspace) + align_up(p.records_bytes);
    j.gb.chunk_start = reinterpret_cast<uint32_t *>(tables);
    j.gb.tile_start = reinterpret_cast<uint32_t *>(tables + align_up(p.table_bytes));
    j.gb.tile_sums = reinterpret_cast<uint32_t *>(tables + 2 * align_up(p.table_bytes));
    j.gb.n_rb = p.n_rb;
    j.gb.n_chunks = no_splats ? 0 : p.n_chunks;
    j.gb.flushes = p.flushes;
    j.gb.n_tiles = p.n_tiles;
    j.ck.ckpt = ckpt ? ckpt + 2 * static_cast<size_t>(done) : nullptr;
    j.ck.every = ckpt_every;
    j.ck.stride = run->n_points;
    if (no_splats && !ckpt) continue;
    rc = device_status(launch_splat_forward(j, s), "cfs_splat");
    if (rc) return rc;
  }
  return CFS_OK;
}

namespace {

// Backward workspace layout: the gradient partials of every sweep workgroup
// of the run, then, reused by every launch slice, the slice's records, the
// record index of each of its splats (pos), the two run tables, their column
// sums and the splat gradients S (in record order).
struct BwdLayout {
  size_t partials, records, pos, table, sums, s, total;
};

BwdLayout bwd_layout(const cfs_system *sys, const cfs_run *run, const cfs_image *img) {
  BwdLayout l{};
  const uint32_t blocks = (run->n_points + kGBwdBlock - 1) / kGBwdBlock;
  const int ng = sys->n_maps <= 4 ? 4 : 8;
  l.partials = align_up(static_cast<size_t>(std::max<uint32_t>(blocks, 1)) * ng * 6 * sizeof(float));
  if (run->n_iters > run->burn_in && run->n_points > 0) {
    const uint32_t slice = gauss_slice(run);
    const GaussPlan p = gauss_plan(slice, run->n_iters, run->burn_in, img->width, img->height);
    l.records = align_up(p.records_bytes);
    l.pos = align_up(static_cast<size_t>(slice) * (run->n_iters - run->burn_in) * sizeof(uint32_t));
    l.table = align_up(p.table_bytes);
    l.sums = align_up(p.sums_bytes);
    l.s = align_up(p.records_bytes);
  }
  l.total = l.partials + l.records + l.pos + 2 * l.table + l.sums + l.s;
  return l;
}

}  // namespace

extern "C" size_t cfs_splat_backward_workspace(const cfs_system *sys, const cfs_run *run,
                                               const cfs_image *img, float sigma_px) {
  if (validate_gauss(sys, run, img, sigma_px)) return 0;
  return bwd_layout(sys, run, img).total;
}

extern "C" int cfs_splat_backward(const cfs_system *sys, const cfs_run *run, const cfs_image *img,
                                  float sigma_px, const float *dL_dD, const float *ckpt,
                                  int32_t ckpt_every, float *grad, void *workspace,
                                  size_t workspace_bytes, void *stream) {
  clear_error();
  int rc = validate_gauss(sys, run, img, sigma_px);
  if (rc) return rc;
  if (sys->n_maps > 8) return fail(CFS_E_UNSUPPORTED, "the adjoint handles systems of at most 8 maps");
  if (!dL_dD || !ckpt || !grad) return fail(CFS_E_INVALID, "dL_dD, ckpt and grad are required");
  if (ckpt_every < 1 || ckpt_every > kMaxSeg)
    return fail(CFS_E_INVALID, "ckpt_every must be in 1..%d", kMaxSeg);
  if ((reinterpret_cast<uintptr_t>(dL_dD) | reinterpret_cast<uintptr_t>(grad)) % 4 ||
      reinterpret_cast<uintptr_t>(ckpt) % 8)
    return fail(CFS_E_INVALID, "misaligned dL_dD, ckpt or grad");
  const BwdLayout l = bwd_layout(sys, run, img);
  if (!workspace || workspace_bytes < l.total)
    return fail(CFS_E_WORKSPACE, "cfs_splat_backward needs %zu bytes of workspace, got %zu",
                l.total, workspace ? workspace_bytes : static_cast<size_t>(0));
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(CFS_E_WORKSPACE, "workspace must be 256-byte aligned");
  GaussJob job;
  std::memset(&job, 0, sizeof job);
  rc = pack_table<2>(sys, &job.mt, &job.equal);
  if (rc) return rc;
  job.gp = make_gauss_params(run, img, sigma_px);
  job.dLdD = dL_dD;
  job.grad = grad;
  char *ws = static_cast<char *>(workspace);
  job.partials = reinterpret_cast<float *>(ws);
  char *p = ws + l.partials;
  job.gb.records = reinterpret_cast<float2 *>(p);
  job.gb.pos = reinterpret_cast<uint32_t *>(p + l.records);
  job.gb.chunk_start = reinterpret_cast<uint32_t *>(p + l.records + l.pos);
  job.gb.tile_start = reinterpret_cast<uint32_t *>(p + l.records + l.pos + l.table);
  job.gb.tile_sums = reinterpret_cast<uint32_t *>(p + l.records + l.pos + 2 * l.table);
  job.S = reinterpret_cast<float2 *>(p + l.records + l.pos + 2 * l.table + l.sums);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (run->n_iters == run->burn_in || run->n_points == 0) {
    // nothing is splatted: the density, hence the loss, does not depend on
    // the maps and the gradient is exactly zero (+0.0f is the all-zero word)
    return device_status(launch_clear_u32(reinterpret_cast<uint32_t *>(grad),
                                          static_cast<size_t>(sys->n_maps) * 6, s),
                         "cfs_splat_backward");
  }
  const RunArgs ra = make_run_args(run);
  const bool splats = run->n_iters > run->burn_in;
  const uint32_t slice = gauss_slice(run);
  for (uint32_t done = 0; done < run->n_points; done += slice) {
    const uint32_t pts = std::min(slice, run->n_points - done);
    GaussJob j = job;
    j.ra = ra;
    j.ra.n_points = pts;
    j.ra.point_offset = run->point_offset + done;
    const GaussPlan gpl = gauss_plan(pts, run->n_iters, run->burn_in, img->width, img->height);
    j.gb.n_chunks = splats ? gpl.n_chunks : 0;
    j.gb.flushes = gpl.flushes;
    j.gb.n_tiles = gpl.n_tiles;
    j.gb.n_rb = gpl.n_rb;
    j.ck.ckpt = const_cast<float *>(ckpt) + 2 * static_cast<size_t>(done);
    j.ck.every = ckpt_every;
    j.ck.stride = run->n_points;
    // slices are multiples of the sweep's workgroup size
    rc = device_status(launch_splat_backward_slice(j, done / kGBwdBlock, s), "cfs_splat_backward");
    if (rc) return rc;
  }
  const uint32_t blocks = (run->n_points + kGBwdBlock - 1) / kGBwdBlock;
  return device_status(launch_grad_reduce(job, blocks, s), "cfs_splat_backward");
}

extern "C" size_t cfs_l2_loss_workspace(uint64_t n) {
  return static_cast<size_t>(loss_blocks(n)) * sizeof(double);
}

extern "C" int cfs_l2_loss(const float *density, const float *target, uint64_t n, float *dL_dD,
                           double *loss, void *workspace, size_t workspace_bytes, void *stream) {
  clear_error();
  if (!loss) return fail(CFS_E_INVALID, "loss is NULL");
  if (n && (!density || !target)) return fail(CFS_E_INVALID, "density/target is NULL");
  if (n > (1ull << 40)) return fail(CFS_E_INVALID, "n exceeds 2^40");
  const size_t need = cfs_l2_loss_workspace(n);
  if (!workspace || workspace_bytes < need)
    return fail(CFS_E_WORKSPACE, "cfs_l2_loss needs %zu bytes of workspace, got %zu", need,
                workspace ? workspace_bytes : static_cast<size_t>(0));
  if (reinterpret_cast<uintptr_t>(workspace) % 8 || reinterpret_cast<uintptr_t>(loss) % 8)
    return fail(CFS_E_INVALID, "workspace and loss must be 8-byte aligned");
  return device_status(launch_l2_loss(density, target, n, dL_dD, loss,
                                      static_cast<double *>(workspace),
                                      static_cast<hipStream_t>(stream)),
                       "cfs_l2_loss");
}
