// vqs_learned.hip -- learned splitter: placeholder until the model kernels land.
#include "vqs_learned.h"

namespace vqs {

void LearnedState::release() {
  if (mem) (void)hipFree(mem);
  mem = nullptr;
  bytes = 0;
}

void LearnedState::fill_stats(vqs_stats* out) const {
  if (!valid) return;
  out->learned_buckets = last.learned_buckets;
  out->overflow_buckets = last.overflow_buckets;
  out->max_bucket = last.max_bucket;
  out->train_loss = last.train_loss;
}

int learned_sort(LearnedState&, const Params&, uint64_t, const vqs_options*, hipStream_t, int*) {
  return VQS_EINVAL;
}

}  // namespace vqs
