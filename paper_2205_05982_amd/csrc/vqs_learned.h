// vqs_learned.h -- launchers of the learned 256-bucket splitter kernels.
//
// The model is a 1 -> 32 -> 32 -> 1 perceptron with clamp-to-[0,1] activations and
// non-negative weight matrices, read as an approximation of the key distribution's
// CDF over the monotone input map x(k) (the key rounded to float, its bit pattern
// read as an unsigned integer, converted to float, times 2^-31).  Non-negative
// weights and non-decreasing activations make the bucket map
// b(k) = min(255, floor(256 * y(x(k)))) non-decreasing in k, so every key of bucket b
// precedes every key of bucket b+1 and a 256-way partition by b followed by sorting
// each bucket sorts the array.  The map is compiled exactly into thresholds
// t_j = min{k : b(k) >= j}, so classification is a binary search.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vqs {

constexpr int MLP_H = 32;
constexpr int MLP_NPARAM = MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 1153
constexpr int MLP_NBLOCK = MLP_NPARAM + 2;                                      // + x0, xs
constexpr int MLP_W1 = 0, MLP_B1 = 32, MLP_W2 = 64, MLP_B2 = 64 + 1024, MLP_W3 = MLP_B2 + 32,
              MLP_B3 = MLP_W3 + 32, MLP_X0 = MLP_B3 + 1, MLP_XS = MLP_X0 + 1;
constexpr int MLP_MAX_BATCH = 256;     // samples per optimiser step (one workgroup)
#ifndef VQS_LEARN_TILE
#define VQS_LEARN_TILE 8192
#endif
constexpr int LEARN_TILE = VQS_LEARN_TILE;      // keys per histogram / scatter tile
constexpr int CHUNK_TILES = 65536 / LEARN_TILE; // consecutive tiles counted together and scattered by one workgroup
constexpr int NBUCKET = 256;

struct TrainArgs {
  const float* x;         // sample inputs x(k), sorted
  const float* t;         // mid-rank CDF targets
  uint64_t m;             // samples
  uint32_t steps, batch;
  float lr;
  uint64_t seed;          // batch selection
  int sequential;         // batches are consecutive samples instead of random ones
};

hipError_t launch_sample(const uint64_t* keys, uint64_t n, uint64_t* sample, uint64_t chunks, uint64_t seed,
                         hipStream_t s);
hipError_t launch_targets(const uint64_t* sorted, uint64_t m, float* x, float* t, hipStream_t s);
hipError_t launch_init(float* params, uint64_t seed, const float* x, uint64_t m, hipStream_t s);
hipError_t launch_train(float* params, float* moments, const TrainArgs& a, hipStream_t s);
hipError_t launch_gradient(const float* params, const float* x, const float* t, uint32_t m, float* grad,
                           float* loss, hipStream_t s);
hipError_t launch_forward(const float* params, const float* x, uint64_t m, float* y, hipStream_t s);
hipError_t launch_buckets(const float* params, const uint64_t* keys, uint64_t n, int32_t* out, hipStream_t s);
hipError_t launch_thresholds(const float* params, uint64_t* thr, uint32_t* nvalid, hipStream_t s);
hipError_t launch_classify(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                           int32_t* out, hipStream_t s);
hipError_t launch_histogram(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                            uint32_t* hist, uint64_t nchunks, hipStream_t s);
hipError_t launch_scan(uint32_t* hist, uint64_t nchunks, uint64_t* totals, hipStream_t s);
hipError_t launch_offsets(const uint64_t* totals, uint64_t n, float overflow_factor, int64_t* offsets,
                          uint64_t* summary, hipStream_t s);
hipError_t launch_scatter(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                          const uint32_t* hist, uint64_t nchunks, const int64_t* offsets, uint64_t* out,
                          hipStream_t s);

}  // namespace vqs
