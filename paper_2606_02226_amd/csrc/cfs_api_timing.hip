// cfs_api_timing.hip -- measurement hook: HIP events recorded around each
// kernel that cfs_chaos_game launches, so a caller can time the chaos kernel
// on its own stream without a profiler.  Disabled by default; nothing is
// recorded and no event exists until cfs_timing_enable(1).
#include <array>
#include <mutex>
#include <vector>

#include "cfs.h"
#include "cfs_api_internal.hpp"

namespace cfs {

namespace {

constexpr int kMaxTimedCalls = 256;

struct TimingState {
  std::mutex mu;
  bool enabled = false;
  std::vector<std::array<hipEvent_t, kPhaseEvents>> free;        // created, unused
  std::vector<std::vector<std::array<hipEvent_t, kPhaseEvents>>> calls;  // per call, per slice
};

TimingState &state() {
  static TimingState s;
  return s;
}

}  // namespace

bool timing_begin_call() {
  TimingState &t = state();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.enabled || t.calls.size() >= static_cast<size_t>(kMaxTimedCalls)) return false;
  t.calls.emplace_back();
  return true;
}

const hipEvent_t *timing_slice() {
  TimingState &t = state();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.enabled || t.calls.empty()) return nullptr;
  std::array<hipEvent_t, kPhaseEvents> ev;
  if (!t.free.empty()) {
    ev = t.free.back();
    t.free.pop_back();
  } else {
    for (int i = 0; i < kPhaseEvents; ++i) {
      if (hipEventCreate(&ev[i]) != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
        return nullptr;
      }
    }
  }
  t.calls.back().push_back(ev);
  return t.calls.back().back().data();
}

}  // namespace cfs

using namespace cfs;

extern "C" int cfs_timing_enable(int32_t enable) {
  clear_error();
  TimingState &t = state();
  std::lock_guard<std::mutex> lock(t.mu);
  t.enabled = enable != 0;
  return CFS_OK;
}

extern "C" int cfs_timing_read(float *ms, int32_t max_calls, int32_t *n_calls) {
  clear_error();
  if (!n_calls || (max_calls > 0 && !ms)) return fail(CFS_E_INVALID, "ms/n_calls is NULL");
  TimingState &t = state();
  std::lock_guard<std::mutex> lock(t.mu);
  int32_t n = 0;
  int rc = CFS_OK;
  for (auto &call : t.calls) {
    float sum[kPhaseEvents - 1] = {0.0f, 0.0f, 0.0f};
    for (auto &ev : call) {
      for (int p = 0; p + 1 < kPhaseEvents && rc == CFS_OK; ++p) {
        float v = 0.0f;
        hipError_t e = hipEventSynchronize(ev[p + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&v, ev[p], ev[p + 1]);
        if (e != hipSuccess) rc = device_status(e, "cfs_timing_read");
        sum[p] += v;
      }
      t.free.push_back(ev);
    }
    if (n < max_calls)
      for (int p = 0; p + 1 < kPhaseEvents; ++p) ms[n * (kPhaseEvents - 1) + p] = sum[p];
    ++n;
  }
  t.calls.clear();
  *n_calls = n < max_calls ? n : max_calls;
  return rc;
}
