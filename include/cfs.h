/*
 * cfs.h -- C ABI of the MI355X (gfx950) chaos-game library for composable
 * function systems (CFS).
 *
 * What the library computes (Schloss, "Composable function systems as a
 * general-purpose rendering framework"):
 *   - Section 1, Section 3 (opening): the chaos game.  Many independent points
 *     each start at a random position; every step a point picks one function
 *     of the system at random, applies it, and is then histogrammed (splatted)
 *     onto the output image.
 *   - Section 1 (fig. "workflow"): splats may be coloured by the index of the
 *     function that moved the point.
 *   - Section 3 (fig. "circle" B) and the caption of fig. "workflow": a
 *     composed spatial transform acts on a COPY of the point before it is
 *     splatted; the original keeps iterating.
 *   - Section 1: only the output image and a few bytes of function arguments
 *     live in device memory; no point cloud is stored.
 *   - Section 4 (limitations): density estimation needs atomic operations;
 *     automatic generation of the primitive's distribution is suggested with
 *     tools similar to automatic differentiation -- the Gaussian splat and
 *     its adjoint below are that differentiable form.
 *
 * Conventions shared by every entry point
 *   - Host structs are read only during the call; everything the GPU needs
 *     is copied into kernel arguments or into library-owned device memory.
 *   - Every device pointer is owned by the caller and must stay valid until
 *     the work enqueued on `stream` has finished.  `stream` is a hipStream_t
 *     passed as void*; NULL means the default stream of the current device.
 *   - Work is enqueued asynchronously on `stream`; results are visible after
 *     the caller synchronises that stream.
 *   - Every argument is validated on the host before anything is enqueued:
 *     on error nothing is written and a negative CFS_E_* code is returned;
 *     cfs_last_error() then describes the problem (thread-local string).
 *     Asynchronous device faults surface as CFS_E_DEVICE from a later call.
 *   - Images are planar, row-major: [channels][height][width]; row 0 is at
 *     lo[1], column 0 at lo[0].  A point q lands in pixel
 *     (floor((q.x - lo.x) W / (hi.x - lo.x)), floor((q.y - lo.y) H / (hi.y - lo.y)))
 *     if both are inside [0, W) x [0, H); otherwise (or if NaN) it is dropped.
 *   - Random streams: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed low word, seed high word) and counter (global point id, block,
 *     instance, tag).  Tag 1 block 0 gives the initial point, one 24-bit
 *     word per coordinate on the 2^-24 grid of [0,1)^dim; tag 0 block j gives
 *     the four draws of iterations 4j+1 .. 4j+4.  The draw u of an iteration
 *     selects map k = min{ i : u < thresh[i] } with thresh[i] =
 *     ceil(2^32 P_i) for the FP64 cumulative probabilities P_i (last = 2^32),
 *     or thresh[i] = ceil((i+1) 2^32 / n) when prob is NULL.  Because the
 *     streams are keyed by global point id, runs split by point ranges add up
 *     exactly to the whole run.
 */
#ifndef CFS_H
#define CFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFS_VERSION 1

/* Status codes. */
#define CFS_OK 0
#define CFS_E_INVALID (-1)     /* an argument failed validation */
#define CFS_E_UNSUPPORTED (-2) /* valid but not implemented combination */
#define CFS_E_NOMEM (-3)       /* a library-owned allocation failed */
#define CFS_E_DEVICE (-4)      /* the HIP runtime reported an error */
#define CFS_E_WORKSPACE (-5)   /* workspace missing or too small */

#define CFS_MAX_MAPS 64

/* Composed transform applied to the copy of the point before splatting. */
enum {
  CFS_FINAL_IDENTITY = 0,     /* q = (p.x, p.y) */
  CFS_FINAL_SWIRL = 1,        /* 2D, params {cx, cy, kappa, tx, ty}:
                                 d = p - c, r = |d|, q = c + t + R(kappa r) d */
  CFS_FINAL_TWIST_CAMERA = 2, /* 3D, params {kappa, cx, cy, cz, M[12], fx, fy}:
                                 w = p - c twisted about the vertical axis by
                                 kappa w.y, v = M[:, :3] w + M[:, 3],
                                 q = (fx v.x / v.z, fy v.y / v.z), depth v.z */
  CFS_FINAL_STRETCH = 3,      /* 2D, params {sx, sy}: q = (sx x, y - sy cos x)
                                 (Section 3's stretch is sx = 2, sy = 1) */
  CFS_FINAL_RING = 4          /* 2D, params {r_in, r_out}: the point at radius
                                 r about the origin moves along its ray to
                                 radius sqrt(r_in^2 + (r_out^2 - r_in^2) r^2)
                                 (the origin to (r_in, 0)): the uniform unit
                                 disk becomes the uniform annulus, the rings
                                 of Section 3's multiple-objects scene */
};

/* Image element types. */
enum {
  CFS_IMAGE_U32_COUNT = 0,   /* uint32 [channels][H][W]; channels 1 or n_maps
                                (then channel = index of the last map) */
  CFS_IMAGE_F32_DENSITY = 1, /* float  [H][W] */
  CFS_IMAGE_U64_DEPTH = 2    /* uint64 [H][W] min of (float bits of depth) << 32
                                | map index, plus uint32 density [H][W] */
};

/* Arithmetic type of the point positions and transforms on the GPU. */
enum { CFS_PREC_F32 = 0, CFS_PREC_F64 = 1 };

/* How integer splats (counts, depth keys) reach the image.  DIRECT: device
 * atomics per splat.  BINNED: each workgroup sorts its splats by image tile
 * in LDS and writes them out as per-tile runs; a second kernel accumulates
 * every tile in LDS and merges it into the image (needs workspace; count
 * images of at most 2^25 elements, depth images of at most 2^24 pixels).
 * One workgroup's records must fit one launch's record budget (2^29 16-bit
 * count records or 2^30 8-byte depth records), which holds about 10^6
 * splatted steps per point;
 * longer runs take DIRECT under AUTO and are refused
 * (CFS_E_UNSUPPORTED) under BINNED.  AUTO picks BINNED for large runs that
 * qualify.  Both give bit-identical images (integer sums and minima do not
 * depend on order). */
enum { CFS_SPLAT_AUTO = 0, CFS_SPLAT_DIRECT = 1, CFS_SPLAT_BINNED = 2 };

/* How the composed transform meets the iteration (Section 3, fig. "circle"
 * B vs C): COPY transforms a copy of the point before the splat and keeps
 * iterating the original; REUSE feeds the transformed point back, so the
 * iterated maps are the transform composed with each map (2D transforms
 * only, count images only). */
enum { CFS_COMPOSE_COPY = 0, CFS_COMPOSE_REUSE = 1 };

/* Kinds of the maps of a system. */
enum {
  CFS_MAP_AFFINE = 0, /* p -> A_k p + b_k */
  CFS_MAP_CIRCLE = 1  /* 2D, the circle map of Section 3's circle equation,
                         read as: u = |p|^2, v = (polar angle in [0, 2 pi))
                         / (2 pi); the image has radius sqrt(v) and angle
                         pi (u + f) with f = b_k[0] (the map's id, 0 or 1);
                         it keeps the uniform disk and sends it onto its
                         upper (f = 0) or lower (f = 1) half; A_k unused */
};

/* A function system: n maps (affine unless `kind` says otherwise) and a
 * composed transform.  The map table is copied into kernel arguments (a few
 * KiB at most). */
typedef struct cfs_system {
  int32_t dim;            /* 2 or 3 */
  int32_t n_maps;         /* 1 .. CFS_MAX_MAPS */
  const float *A;         /* host [n_maps][dim][dim], row-major */
  const float *b;         /* host [n_maps][dim] */
  const double *prob;     /* host [n_maps] summing to 1 (+-1e-6), or NULL */
  int32_t final_kind;     /* CFS_FINAL_* */
  float final_params[24]; /* meaning per final_kind, unused entries ignored */
  const int32_t *kind;    /* host [n_maps] CFS_MAP_*, or NULL (all affine);
                             circle maps need dim 2 */
  int32_t compose;        /* CFS_COMPOSE_COPY (default) or CFS_COMPOSE_REUSE */
} cfs_system;

/* One run over a range of points.
 * Continued runs (cfs_chaos_game only; Section 3: a point's chaos game is
 * one sequence of steps, so it can be cut into calls): with iter_offset
 * K > 0 every point has already taken K steps, its position after them is
 * read from final_points (which must be given, in the run's precision) and
 * overwritten with its position after this call's T further steps; step t
 * of the call is step K + t of the game (map draw: word (K + t - 1) mod 4
 * of Philox block (K + t - 1) / 4), and burn_in counts the game's steps, so
 * a call inside the burn-in splats nothing.  K must be a multiple of 4 (the
 * kernels draw whole Philox blocks).  A game cut into calls this way gives
 * the same indices, positions and (summed) image as one call. */
typedef struct cfs_run {
  uint64_t seed;          /* Philox key */
  uint32_t instance;      /* third counter word (batched instance id) */
  uint32_t n_points;      /* N */
  uint32_t point_offset;  /* global id of the first point; offset + N <= 2^32 */
  uint32_t n_iters;       /* T map applications per point, 1 .. 2^20 */
  uint32_t burn_in;       /* B: steps 1..B of the game are not splatted (B <= T
                             except in cfs_chaos_game) */
  int32_t precision;      /* CFS_PREC_F32 or CFS_PREC_F64 */
  int32_t splat_path;     /* CFS_SPLAT_AUTO / _DIRECT / _BINNED (count images) */
  uint32_t iter_offset;   /* K: steps already taken (0 = a fresh game); a
                             multiple of 4, at most 2^30 */
} cfs_run;

/* An output image in device memory. */
typedef struct cfs_image {
  int32_t kind;           /* CFS_IMAGE_* */
  int32_t width, height;  /* 1 .. 65536 each; W*H*channels <= 2^31 */
  int32_t channels;       /* 1, or n_maps for per-index counts */
  float lo[2], hi[2];     /* window, lo < hi */
  float near_plane;       /* depth images: splats with depth <= near dropped;
                             must be >= 0 (keys order depths by their FP32
                             bits, which is their order only when >= 0) */
  void *data;             /* device, element type per kind (see above) */
  uint32_t *density;      /* device uint32 [H][W], CFS_IMAGE_U64_DEPTH only */
  unsigned long long *dropped; /* device counter of dropped splats, or NULL */
} cfs_image;

/* Library version (CFS_VERSION). */
int cfs_version(void);

/* Description of the last error on the calling thread ("" if none). */
const char *cfs_last_error(void);

/* Image initialisation (the image is the method's only global allocation,
 * Section 1): counts and densities to 0, depth keys to all ones, density of a
 * depth image to 0, and *dropped to 0.  Enqueued on `stream`. */
int cfs_image_clear(const cfs_image *img, void *stream);

/* Workspace in bytes that cfs_chaos_game needs for this system, run and
 * image (0 when the direct-atomic splat is used).  Returns 0 on invalid
 * arguments as well; cfs_chaos_game then reports the error. */
size_t cfs_chaos_game_workspace(const cfs_system *sys, const cfs_run *run,
                                const cfs_image *img);

/* The plain chaos game with an integer splat (Section 1, Section 3):
 * for each of run->n_points points, iterate run->n_iters maps chosen from
 * the point's own random stream and, after burn-in, splat the transformed
 * copy (final_kind) into `img`, which ACCUMULATES (the caller clears it,
 * e.g. with cfs_image_clear), so point-range splits compose exactly.
 *   img->kind CFS_IMAGE_U32_COUNT: +1 per splat (channel = last map index
 *     when channels == n_maps); CFS_IMAGE_U64_DEPTH (3D, TWIST_CAMERA):
 *     atomic min of the depth|index key and +1 in img->density.
 *   final_points: device, nullable; [n_points][dim] of float (F32) or
 *     double (F64): each point's position after n_iters steps.
 *   last_index:   device, nullable; uint8 [n_points]: index of the last map.
 *   indices:      device, nullable; uint8 [n_points][n_iters]: every index.
 *   workspace:    device scratch, 256-byte aligned; contents need no
 *     initialisation.  cfs_chaos_game_workspace() bytes give the fewest
 *     launches (may be NULL when that is 0); a smaller workspace cuts the
 *     binned splat into more point-range launches that fit it (the same
 *     result), down to one workgroup's records; below that CFS_SPLAT_AUTO
 *     takes the direct splat and CFS_SPLAT_BINNED fails with
 *     CFS_E_WORKSPACE.
 * Returns CFS_OK or a negative CFS_E_* code (nothing enqueued on error). */
int cfs_chaos_game(const cfs_system *sys, const cfs_run *run,
                   const cfs_image *img, void *final_points,
                   uint8_t *last_index, uint8_t *indices, void *workspace,
                   size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): the same
 * chaos game as cfs_chaos_game, same arguments and results, with the
 * binned splat's records and run tables in a fixed array of
 * CFS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * (until the process ends) instead of a caller workspace.  A binned run is
 * cut into point-range launches whose records and tables fit that array
 * (the result is the same: the random streams are keyed by point id).
 * A run whose single workgroup of points does not fit (from about 6 x 10^4
 * splatted steps per point for depth images to 2.6 x 10^5 for small count
 * images) takes the direct splat under CFS_SPLAT_AUTO and fails
 * with CFS_E_UNSUPPORTED under CFS_SPLAT_BINNED.  Calls no hipMalloc or
 * hipFree; the first call on a device looks up that device's array (the
 * stream must belong to the current device).  Every call on one GPU shares
 * its array, which keeps the last call's contents (nothing in it needs
 * clearing): calls that overlap on one GPU -- concurrent streams or host
 * threads -- race and must be serialised by the caller.  The measurement
 * hook does not time these calls. */
#define CFS_NOALLOC_SCRATCH_BYTES (256ull << 20)
int cfs_chaos_game_noalloc(const cfs_system *sys, const cfs_run *run,
                           const cfs_image *img, void *final_points,
                           uint8_t *last_index, uint8_t *indices, void *stream);

/* Measurement hook.  While enabled, every cfs_chaos_game call (up to 256
 * calls between reads) records HIP events on its stream before its chaos
 * kernel, after it, after the run-table transpose and after the tile
 * accumulate (binned path; the last two phases are empty for the direct
 * path), so a caller can time the chaos kernel alone on the stream it runs
 * on.  Enabling costs four event records per launch slice and no device
 * memory.  Default: off. */
int cfs_timing_enable(int32_t enable);

/* Waits for the recorded events and writes, for each recorded call i in
 * call order (i < max_calls), the milliseconds of its phases summed over its
 * launch slices: ms[3 i + 0] chaos kernel, ms[3 i + 1] transpose,
 * ms[3 i + 2] accumulate (host float array of 3 * max_calls).  *n_calls gets
 * the number of entries written; the record is then cleared. */
int cfs_timing_read(float *ms, int32_t max_calls, int32_t *n_calls);

/* Workspace in bytes that cfs_splat needs for this system, run and image. */
size_t cfs_splat_workspace(const cfs_system *sys, const cfs_run *run,
                           const cfs_image *img, float sigma_px);

/* Several objects from one primitive (Section 3, multiple objects from a
 * single primitive; fig. "space"): after every step of the chaos game the
 * point is repositioned once per object and each object's copy is splatted;
 * the point itself keeps iterating.  An object is a 2D transform
 * (final_kind IDENTITY, SWIRL, STRETCH or RING with its final_params), then
 * the placement q' = P q + t (place = a00 a01 a10 a11 t0 t1), then, for
 * n_copies > 1, duplication: each splat goes to one copy c drawn from the
 * point's random stream, and copy c is scaled and moved by values that the
 * random stream of c alone gives, so no copy table exists anywhere:
 *   draw of iteration t: word (t-1) mod 4 of Philox block
 *     (point id, (t-1)/4, instance, 2); object o takes
 *     c = floor(((2o + 1) u mod 2^32) n_copies / 2^32);
 *   copy c of object o: Philox block (c, o, instance, 3), e_i = (w_i >> 8)
 *     2^-24; q'' = (scale_lo + scale_span e_2) q' + copy_lo + copy_span e_{0,1}.
 * Each object splats +1 into channel `channel` of a U32_COUNT image. */
#define CFS_MAX_OBJECTS 8

typedef struct cfs_object {
  int32_t final_kind;      /* CFS_FINAL_IDENTITY, _SWIRL, _STRETCH or _RING */
  float final_params[24];  /* as for cfs_system.final_params */
  float place[6];          /* P row-major, then t */
  int32_t channel;         /* 0 .. image channels - 1 */
  uint32_t n_copies;       /* 1 (no duplication) .. 2^24 */
  float copy_lo[2];        /* offset of copy c: copy_lo + copy_span e */
  float copy_span[2];
  float scale_lo;          /* scale of copy c: scale_lo + scale_span e_2 */
  float scale_span;
} cfs_object;

/* Workspace in bytes for cfs_chaos_scene (0 for the direct splat). */
size_t cfs_chaos_scene_workspace(const cfs_system *sys, const cfs_object *objects,
                                 int32_t n_objects, const cfs_run *run,
                                 const cfs_image *img);

/* The chaos game of a 2D primitive (sys: dim 2, final_kind IDENTITY, compose
 * COPY; affine or circle maps) splatted through n_objects (1..8) objects
 * into the U32_COUNT image img, which ACCUMULATES; *img->dropped (if given)
 * counts splats outside the window.  run->precision and run->splat_path as
 * for cfs_chaos_game; workspace as cfs_chaos_scene_workspace() says (256-byte
 * aligned). */
int cfs_chaos_scene(const cfs_system *sys, const cfs_object *objects, int32_t n_objects,
                    const cfs_run *run, const cfs_image *img, void *workspace,
                    size_t workspace_bytes, void *stream);

/* Differentiable form, forward (Section 4: automatic generation of the
 * primitive's distribution with autodiff-like tools): the chaos game of a 2D
 * affine system with the identity transform, FP32 positions, splatted with
 * the separable shifted-truncated Gaussian
 *   g(d) = exp(-d^2 / (2 s^2)) - exp(-9/2) for |d| < 3 s, else 0
 * (s = sigma_px; d = pixel centre - point, in pixels; pixel (i, j) gets
 * g(i + 0.5 - x) g(j + 0.5 - y); taps off the image are skipped) into the
 * FP32 density img (kind CFS_IMAGE_F32_DENSITY, one channel), which
 * ACCUMULATES sum(w) / (N (T - B)).  The records of an image tile are summed
 * by several workgroups, each over its share of C records: each tap weight is
 * rounded to a multiple of 2^-s with s = 32 - bit length of C (2^-21 for the
 * usual shares of up to 2047 records; C taps then fit 32 bits) and summed
 * exactly; the workgroups' sums are added in FP32 in no fixed order, so
 * results agree with any other order up to rounding.
 *   ckpt: device, nullable; float [ceil(n_iters / ckpt_every)][n_points][2]:
 *     positions at iterations 0, c, 2c, ... (c = ckpt_every in 1..16), from
 *     which cfs_splat_backward recomputes its segments (written also when
 *     burn_in == n_iters, where nothing is splatted).
 *   workspace: device, cfs_splat_workspace() bytes, 256-byte aligned.
 * sigma_px in (0, 2.5]. */
int cfs_splat(const cfs_system *sys, const cfs_run *run, const cfs_image *img,
              float sigma_px, float *ckpt, int32_t ckpt_every, void *workspace,
              size_t workspace_bytes, void *stream);

/* Workspace in bytes for cfs_splat_backward with this system, run, density
 * image and sigma (0 on invalid arguments). */
size_t cfs_splat_backward_workspace(const cfs_system *sys, const cfs_run *run,
                                    const cfs_image *img, float sigma_px);

/* Differentiable form, adjoint: given dL/dD (device float [H][W], the
 * upstream gradient of the density that cfs_splat produced) and that call's
 * checkpoints, recompute each trajectory segment and run the adjoint
 *   lam_T = s_T, lam_t = s_t + A_{k_{t+1}}^T lam_{t+1},
 *   dL/dA_{k_t} += lam_t p_{t-1}^T, dL/db_{k_t} += lam_t
 * (s_t = dL/dp_t through the splat of step t; zero for t <= B).
 * grad (device float [n_maps][6] = a00 a01 a10 a11 b0 b1) is OVERWRITTEN;
 * the reduction is deterministic (per-lane sums, a fixed-order tree per
 * workgroup, and a fixed-order two-level FP64 sum over workgroups; no
 * floating-point atomics).  ckpt must be
 * the forward's checkpoints for the same system, run and ckpt_every (1..16).
 * The splat gradients s_t are computed per image tile from an LDS copy of
 * dL/dD over the splats' records (recomputed from the random streams), then
 * each point's sweep reads them.  workspace: device,
 * cfs_splat_backward_workspace() bytes, 256-byte aligned.
 * With burn_in == n_iters (no splats) or no points the gradient is exactly
 * zero and nothing else is read.  Systems of at most 8 maps. */
int cfs_splat_backward(const cfs_system *sys, const cfs_run *run,
                       const cfs_image *img, float sigma_px,
                       const float *dL_dD, const float *ckpt,
                       int32_t ckpt_every, float *grad, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Workspace in bytes for cfs_l2_loss over n elements. */
size_t cfs_l2_loss_workspace(uint64_t n);

/* Image loss of the fitting loop (Section 4: fitting a primitive's
 * distribution with autodiff-like tools): with D = density and D* = target
 * (device float [n] each),
 *   *loss  = sum_i (D_i - D*_i)^2     (device double, FP64 sum), and
 *   dL_dD_i = 2 (D_i - D*_i)          (device float [n], nullable),
 * the upstream gradient that cfs_splat_backward takes.  The reduction has a
 * fixed order for a given n, so the loss is bit-reproducible.  workspace:
 * device, cfs_l2_loss_workspace(n) bytes, 8-byte aligned; loss 8-byte
 * aligned. */
int cfs_l2_loss(const float *density, const float *target, uint64_t n, float *dL_dD,
                double *loss, void *workspace, size_t workspace_bytes, void *stream);

/* Batched form: many heterogeneous systems (animation frames, different map
 * counts, point counts and image sizes) rendered by persistent kernels inside
 * ONE HIP graph launch (abstract and Section 4 of the paper: animation).  Each
 * instance renders exactly what cfs_chaos_game renders for it (same random
 * streams, same device functions, FP32 or FP64 positions per instance), so
 * its image is bit-identical to the plain call's. */
typedef struct cfs_batch_item {
  cfs_system sys;  /* 2D, affine maps, identity transform, up to CFS_MAX_MAPS
                      maps */
  cfs_run run;     /* run.instance selects the instance's random streams;
                      splat_path is ignored (the plan decides) */
  cfs_image img;   /* CFS_IMAGE_U32_COUNT, 1 or n_maps channels, caller-owned
                      data that must stay valid while the batch exists */
} cfs_batch_item;

/* Schedule of a batch.  blocks_per_item: 512-point blocks per work item
 * popped from the device queue (>= 1); emit_grid: persistent workgroups of
 * the chaos kernels (0 = two per compute unit); acc_grid: persistent
 * workgroups of the tile-accumulate kernel (0 = two per compute unit);
 * splat_path: CFS_SPLAT_BINNED or CFS_SPLAT_DIRECT (CFS_SPLAT_AUTO = binned);
 * direct_below: the per-instance strategy of a BINNED plan -- an instance
 * with fewer than direct_below splats (points x splatted steps) takes the
 * direct splat (device atomics; no records, run tables or accumulate items),
 * the others the binned splat (0 = every instance binned). */
typedef struct cfs_plan {
  int32_t blocks_per_item;
  int32_t emit_grid;
  int32_t acc_grid;
  int32_t splat_path;
  uint64_t direct_below;
} cfs_plan;

typedef struct cfs_batch cfs_batch; /* opaque, library-owned */

/* Build a batch on the current device: copies the descriptors into
 * library-owned device memory, lays out the work queues (one item per
 * blocks_per_item blocks of an instance; one accumulate item per image tile)
 * and allocates the records of the binned splat.  plan NULL = defaults
 * (blocks_per_item 4, both grids two per compute unit, binned; use
 * cfs_autotune to pick one).  *out receives the handle. */
int cfs_batch_create(const cfs_batch_item *items, int32_t n_items,
                     const cfs_plan *plan, cfs_batch **out);

/* Enqueue the whole batch on `stream`: clear every image, reset the work
 * queues, run the persistent chaos kernel and the persistent accumulate
 * kernel.  The first call captures these into a HIP graph (on a library
 * stream); every call launches that graph on `stream`.  Calls on one batch
 * must not overlap (they share the queues and records). */
int cfs_batch_run(cfs_batch *batch, void *stream);

/* Replace instance `index`'s map table and probabilities (same map count;
 * e.g. the next animation frame) without re-capturing the graph.  The new
 * table is written by a kernel ordered on `stream`. */
int cfs_batch_update(cfs_batch *batch, int32_t index, const cfs_system *sys,
                     void *stream);

/* The plan a batch uses. */
int cfs_batch_plan(const cfs_batch *batch, cfs_plan *out);

/* Free the batch (waits for the device to finish its work first). */
void cfs_batch_destroy(cfs_batch *batch);

/* Project-written autotuner: builds the batch with each candidate plan (both
 * splat paths, several work-item sizes and accumulate grids; then, for the
 * fastest binned shape, several per-instance thresholds direct_below), times
 * graph replays with HIP events on `stream`, and writes the fastest plan to
 * *out.  The images are overwritten by the trial runs.
 *   cache_path: host, nullable; a JSON Lines file of tuned plans keyed by
 *     (device architecture name, compute units, signature of the batch's
 *     shapes: per instance map count, equal or not, points, iterations,
 *     burn-in, image size and channels, precision).  A matching line is
 *     returned without timing anything (and without touching the images);
 *     otherwise the tuned plan is appended as a new line.  An unreadable or
 *     unwritable file is treated as empty / skipped. */
int cfs_autotune(const cfs_batch_item *items, int32_t n_items, cfs_plan *out,
                 const char *cache_path, void *stream);

/* Parity hook: out[i] = Philox4x32-10(ctrs[i], key(seed)) for i < n.
 * ctrs, out: device uint32 [n][4]. */
int cfs_philox_dump(uint64_t seed, const uint32_t *ctrs, uint32_t *out,
                    uint64_t n, void *stream);

/* Ceiling probes for the rooflines (measurement hook).  The splat is an
 * atomic histogram (Section 1; Section 4 names its atomics as a limit), and
 * the chip's atomic rates are not published, so they are measured with the
 * operation types of the splats:
 *   COPY         buf = [src half | dst half]: copy bytes / 2; *done = bytes
 *                moved (read + written);
 *   DEV_ADD_U32  about `ops` u32 atomic adds at uniformly random elements of
 *                the device working set buf (bytes / 4 elements);
 *   DEV_MIN_U64  the same with u64 atomic minima (bytes / 8 elements);
 *   LDS_ADD_U32  about `ops` u32 atomic adds at random words of a 64 KiB LDS
 *                table per 1024-lane workgroup (512 workgroups); buf
 *                receives one word per workgroup (bytes >= 2 KiB);
 *   LDS_MIN_U64  the same with u64 atomic minima (bytes >= 4 KiB);
 *   LDS_ADD_U64  the same with u64 atomic adds (bytes >= 4 KiB);
 *   PHILOX       about `ops` Philox4x32-10 blocks (buf >= 4 MiB receives one
 *                word per lane);
 *   RUNS_128, RUNS_512, RUNS_2048
 *                about `ops` reads of runs of 128, 512 or 2048 bytes at
 *                uniformly random 16-byte-aligned places (8, 32 or 128 lanes
 *                per run, 16 bytes each, four runs in flight per group): the
 *                first 4 MiB of buf receive one word per lane, the rest
 *                holds the runs (make it larger than the caches); *done =
 *                bytes read.
 * buf: device, 16-byte aligned, caller-owned; its contents are overwritten.
 * *done (host) receives the operations (or bytes) actually issued; the
 * caller times the call with events on `stream`.  Enqueues one kernel. */
enum {
  CFS_MB_COPY = 0,
  CFS_MB_DEV_ADD_U32 = 1,
  CFS_MB_DEV_MIN_U64 = 2,
  CFS_MB_LDS_ADD_U32 = 3,
  CFS_MB_LDS_MIN_U64 = 4,
  CFS_MB_PHILOX = 5,
  CFS_MB_LDS_ADD_U64 = 6,
  CFS_MB_RUNS_128 = 7,
  CFS_MB_RUNS_512 = 8,
  CFS_MB_RUNS_2048 = 9
};
int cfs_microbench(int32_t kind, void *buf, size_t bytes, uint64_t ops,
                   uint64_t *done, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CFS_H */
