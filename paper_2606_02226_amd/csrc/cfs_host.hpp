// cfs_host.hpp -- host-side job descriptions passed from the C-ABI layer to
// the kernel launchers (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "cfs_params.hpp"

namespace cfs {

struct FinalArgs {
  float p[24];
};

struct ChaosJob {
  int dim;
  int final_kind;
  int precision;  // 0 = FP32, 1 = FP64
  bool equal;     // equal probabilities
  bool depth;     // U64 depth image (3D camera)
  MapTable<2> mt2;
  MapTable<3> mt3;
  Window win;
  RunArgs ra;
  FinalArgs fa;
  void *img;
  uint32_t *density;
  float near_plane;
  Outputs out;
};

hipError_t launch_chaos(const ChaosJob &job, hipStream_t stream);
hipError_t launch_clear_u32(uint32_t *p, size_t n, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v,
                           hipStream_t stream);
hipError_t launch_philox_dump(uint32_t k0, uint32_t k1, const uint32_t *ctrs,
                              uint32_t *out, uint64_t n, hipStream_t stream);

}  // namespace cfs
