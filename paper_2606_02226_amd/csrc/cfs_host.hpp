// cfs_host.hpp -- host-side job descriptions passed from the C-ABI layer to
// the kernel launchers (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "cfs_params.hpp"

namespace cfs {

constexpr int kFinalParams = 24;
struct FinalArgs {
  float p[kFinalParams];
};

struct ChaosJob {
  int dim;
  int final_kind;
  int precision;  // 0 = FP32, 1 = FP64
  bool equal;     // equal probabilities
  bool depth;     // U64 depth image (3D camera)
  bool binned;    // binned count splat (needs ba)
  MapTable<2> mt2;
  MapTable<3> mt3;
  Window win;
  RunArgs ra;
  FinalArgs fa;
  void *img;
  uint32_t *density;
  float near_plane;
  Outputs out;
  BinArgs ba;
  const hipEvent_t *ev;  // kPhaseEvents events to record around the phases, or null
};

// Records and table sizes of the binned splat for one launch of `points`.
struct BinPlan {
  uint32_t blocks, flushes, n_chunks, n_tiles, elems, parts, log2g, n_rb;
  size_t records_bytes, table_bytes, sums_bytes;
};
// Accumulate launch shape for `records` count records in n_chunks chunks over
// n_tiles tiles, aiming at `target` workgroups: workgroups per tile and lanes
// per run (2^log2g).  bin_plan aims at kAccTargetSkip (its accumulate skips
// tiles without records).
void acc_shape(uint64_t records, uint32_t n_chunks, uint32_t n_tiles, uint32_t target,
               uint32_t *parts, uint32_t *log2g);
// per_iter: records a lane stages per step after burn-in (objects of a scene).
BinPlan bin_plan(uint32_t points, uint32_t n_iters, uint32_t burn_in, uint32_t elems,
                 bool depth = false, uint32_t per_iter = 1);

// Events recorded around the phases of one launch (chaos kernel, table
// transpose, tile accumulate): before, between and after them.
constexpr int kPhaseEvents = 4;
hipError_t launch_chaos_binned(const ChaosJob &job, hipStream_t stream);
// Record event i of a phase-event array on the stream (no-op for null).
inline void mark_phase(const hipEvent_t *ev, int i, hipStream_t s) {
  if (ev) (void)hipEventRecord(ev[i], s);
}
// Transpose the run table and add the binned count records into img.
hipError_t launch_count_accumulate(const BinArgs &ba, uint32_t *img, hipStream_t stream,
                                   const hipEvent_t *ev = nullptr);

struct SceneJob {
  int precision;
  bool equal;
  bool binned;
  MapTable<2> mt;
  Window win;
  RunArgs ra;
  SceneArgs sc;
  uint32_t *img;
  unsigned long long *dropped;
  BinArgs ba;
};
hipError_t launch_scene(const SceneJob &job, hipStream_t stream);
// With `sums`: also the column sums of each 64-row block, [cols][ceil(rows / 64)].
hipError_t launch_transpose(const uint32_t *in, uint32_t *out, uint32_t rows, uint32_t cols,
                            hipStream_t stream, uint32_t *sums = nullptr);
hipError_t launch_transpose(const uint16_t *in, uint16_t *out, uint32_t rows, uint32_t cols,
                            hipStream_t stream, uint32_t *sums = nullptr);

struct GaussJob {
  bool equal;
  MapTable<2> mt;
  RunArgs ra;
  GaussParams gp;
  GaussBin gb;
  GaussCkpt ck;
  float *dens;
  unsigned long long *dropped;
  const float *dLdD;
  float2 *S;  // backward: splat gradients in record order (the slice's records)
  float *partials;
  float *grad;
};

struct GaussPlan {
  uint32_t blocks, flushes, n_chunks, n_tiles;
  int32_t tiles_x, tiles_y;
  uint32_t n_rb;  // 64-chunk blocks of the column sums
  size_t records_bytes, table_bytes, sums_bytes;
};
GaussPlan gauss_plan(uint32_t points, uint32_t n_iters, uint32_t burn_in, int width, int height);
hipError_t launch_splat_forward(const GaussJob &job, hipStream_t stream);
// Backward of one launch slice: its records again (with each splat's record index), the splat
// gradients per tile, then the adjoint sweep writing workgroup partials from
// block_offset on; launch_grad_reduce then sums the partials of all slices.
hipError_t launch_splat_backward_slice(const GaussJob &job, uint32_t block_offset,
                                       hipStream_t stream);
hipError_t launch_grad_reduce(const GaussJob &job, uint32_t blocks, hipStream_t stream);

hipError_t launch_chaos(const ChaosJob &job, hipStream_t stream);
uint32_t loss_blocks(uint64_t n);
hipError_t launch_l2_loss(const float *d, const float *target, uint64_t n, float *grad,
                          double *loss, double *partial, hipStream_t stream);
hipError_t launch_clear_u32(uint32_t *p, size_t n, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v,
                           hipStream_t stream);
hipError_t launch_philox_dump(uint32_t k0, uint32_t k1, const uint32_t *ctrs,
                              uint32_t *out, uint64_t n, hipStream_t stream);

}  // namespace cfs
