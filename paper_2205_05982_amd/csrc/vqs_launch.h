// vqs_launch.h -- host-side launchers of the kernels, one instantiation per key width
// (clear, per-workgroup finish) and per key width and level tile size (seeding,
// planning, pivots, level partitions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vqs_types.h"

namespace vqs {

template <int BITS>
struct Launch {
  static hipError_t clear(const Params& p, hipStream_t s);
  static hipError_t solo(const Params& p, int grid, hipStream_t s);
  // in-place level: the prologue, counting and partition launches
  static hipError_t ip_level(const Params& p, int grid, hipStream_t s);
  static constexpr uint64_t local_buffer_keys() { return (uint64_t)LOCAL_BYTES / (BITS / 8); }
};

template <int BITS, int LI>
struct LaunchLevel {
  static hipError_t seed(const Params& p, const int64_t* offsets, uint64_t nseg, hipStream_t s);
  static hipError_t level(const Params& p, int grid, hipStream_t s);
  static hipError_t pivots(const Params& p, int grid, hipStream_t s);
  static hipError_t plan(const Params& p, int grid, hipStream_t s);
  static constexpr uint64_t level_tile_keys() { return (uint64_t)LEVEL_P * LI * (128 / BITS); }
};

}  // namespace vqs
