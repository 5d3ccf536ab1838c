// context_sort.cpp -- std::sort of the same keys, for context timings next to the
// oracle (test infrastructure: called only by the CPU-baseline leg of the benchmark).
// Not a reference for results: the oracle and the plain definition are.
#include <algorithm>
#include <cstdint>
#include <functional>

namespace {
struct U128 {
  uint64_t lo, hi;
};
template <class T>
void sort_t(void* keys, uint64_t n, int ascending) {
  T* k = static_cast<T*>(keys);
  if (ascending)
    std::sort(k, k + n);
  else
    std::sort(k, k + n, std::greater<T>());
}
}  // namespace

extern "C" int ctx_std_sort(void* keys, uint64_t n, int kt, int ascending) {
  switch (kt) {
    case 1: sort_t<uint16_t>(keys, n, ascending); return 0;
    case 2: sort_t<uint32_t>(keys, n, ascending); return 0;
    case 3: sort_t<uint64_t>(keys, n, ascending); return 0;
    case 5: sort_t<float>(keys, n, ascending); return 0;
    case 6: sort_t<double>(keys, n, ascending); return 0;
    case 4: {
      U128* k = static_cast<U128*>(keys);
      auto lt = [](const U128& a, const U128& b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); };
      if (ascending)
        std::sort(k, k + n, lt);
      else
        std::sort(k, k + n, [&](const U128& a, const U128& b) { return lt(b, a); });
      return 0;
    }
    default: return -2;
  }
}
