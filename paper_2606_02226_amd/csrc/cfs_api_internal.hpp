// cfs_api_internal.hpp -- validation and packing helpers shared by the C-ABI
// translation units of the library.
#pragma once

#include "cfs.h"
#include "cfs_host.hpp"

namespace cfs {

int fail(int code, const char *fmt, ...);
void clear_error();
int device_status(hipError_t e, const char *what);
int make_thresholds(const double *prob, int n, uint64_t *thresh);
int validate_system(const cfs_system *s);
int validate_run(const cfs_run *r);
// Entry points without continued runs: iter_offset 0 and burn_in <= n_iters.
int validate_fresh_run(const cfs_run *r);
// The run as one cfs_chaos_game call sees it: burn_in reduced to the part of
// the game's burn-in that lies in this call's steps.
cfs_run call_run(const cfs_run *r);
int validate_window(const cfs_image *img);
Window make_window(const cfs_image *img, bool by_index);
RunArgs make_run_args(const cfs_run *r);
template <int DIM>
int pack_table(const cfs_system *s, MapTable<DIM> *mt, bool *equal);

// One cfs_chaos_game call, validated and packed: the job, this call's view of
// the run, and for the binned path the points per launch and the workspace
// they need.
struct ChaosCall {
  ChaosJob job;
  cfs_run run;
  uint32_t slice;  // points per binned launch
  uint32_t elems;  // image elements (channels * height * width)
  size_t need;     // workspace bytes of one binned launch
};
// Validate and pack a call (nothing is enqueued).  budget > 0 caps the
// workspace of a binned launch at `budget` bytes.
int chaos_prepare(const cfs_system *sys, const cfs_run *run_in, const cfs_image *img,
                  void *final_points, uint8_t *last_index, uint8_t *indices, size_t budget,
                  ChaosCall *call);
// Enqueue a prepared call with `workspace` (call.need bytes for the binned path).
int chaos_launch(const ChaosCall &call, void *workspace, bool timed, hipStream_t stream);

// Measurement hook (cfs_timing_enable): timing_begin_call() opens the record
// of one cfs_chaos_game call (false when timing is off or full); each launch
// slice then asks timing_slice() for kPhaseEvents events to record (null when
// not timing).
bool timing_begin_call();
const hipEvent_t *timing_slice();

}  // namespace cfs
