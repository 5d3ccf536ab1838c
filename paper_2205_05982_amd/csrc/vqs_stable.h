// vqs_stable.h -- launchers of the stable sort's packing kernels.
//
// Quicksort is not stable (Sec. 5), but becomes so when a unique row number is
// appended to the least-significant bits of each key: the composite keys are all
// distinct and order first by key, then by input position.  pack writes each key's
// order-preserving unsigned form (floats, signed integers and descending order mapped
// as for the sort itself) with its row number; unpack splits the sorted composites
// into keys (transformed back) and rows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vqs {

// Composite layouts: COMP64 = (key << 32) | row as a u64 (16/32-bit keys, n <= 2^32);
// COMP128 = 128-bit key with the key in the high word, the row in the low word.
enum : int { COMP64 = 0, COMP128 = 1 };

hipError_t launch_stable_pack(const void* keys, uint64_t n, int bits, int mode, int comp, void* out,
                              hipStream_t s);
hipError_t launch_stable_unpack(const void* comp_keys, uint64_t n, int bits, int mode, int comp, void* keys,
                                uint64_t* rows, hipStream_t s);

}  // namespace vqs
