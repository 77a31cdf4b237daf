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

// Measurement hook (cfs_timing_enable): timing_begin_call() opens the record
// of one cfs_chaos_game call (false when timing is off or full); each launch
// slice then asks timing_slice() for kPhaseEvents events to record (null when
// not timing).
bool timing_begin_call();
const hipEvent_t *timing_slice();

}  // namespace cfs
