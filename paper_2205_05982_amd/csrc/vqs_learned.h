// vqs_learned.h -- the learned 256-bucket splitter (host side).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/vqs.h"
#include "vqs_types.h"

namespace vqs {

struct LearnedState {
  void* mem = nullptr;
  size_t bytes = 0;
  vqs_stats last{};
  bool valid = false;
  void release();
  void fill_stats(vqs_stats* out) const;
};

// Sort p.keys[0, n) (u64) with the learned splitter in front of the plain method.
int learned_sort(LearnedState& st, const Params& base, uint64_t n, const vqs_options* o, hipStream_t s,
                 int* levels);

}  // namespace vqs
