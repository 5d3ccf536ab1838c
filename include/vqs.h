/*
 * vqs.h -- C interface of the MI355X (gfx950) vectorized Quicksort library.
 *
 * The method is the Quicksort of Blacher, Giesen, Sanders and Wassenberg,
 * "Vectorized and performance-portable Quicksort" (2022): Alg. 1 (recursion with
 * degenerate-partition handling), Sec. 2.1 (Partition: keys not after the pivot
 * move before the others), Sec. 2.2 (ChoosePivot from nine random 64-byte chunks by
 * medians of three; recursion depth limit 2*log2(n)+4 with a bounded-time fallback),
 * Sec. 2.3 and Sec. 3 (BaseCase: 16-row sorting network, Green's column network and
 * transposition-free bitonic merges) and Sec. 2.4 (ascending / descending order,
 * 128-bit keys as pairs of 64-bit halves).
 *
 * Conventions for every entry point:
 *  - keys and offsets are DEVICE pointers owned by the caller (e.g. a torch
 *    tensor's data_ptr()).  Sorting is in place: on return keys holds the result.
 *  - n counts keys, not bytes or words.  keys must be aligned to the key size
 *    (16 bytes for VQS_U128).
 *  - VQS_U128 keys are 16 bytes each, little-endian: the low 64-bit word at byte 0,
 *    the high word at byte 8; they compare as (high, low) lexicographically (Alg. 2).
 *  - Floating-point keys are ordered by the total order of their bit patterns:
 *    -NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN.  For inputs without NaN
 *    and without -0.0 this is the IEEE order, and the result is unique.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL is the default
 *    stream).  Argument errors return at once without launching anything.  The
 *    library keeps a scratch workspace of n keys plus bookkeeping per stream,
 *    allocated on first use and reused; calls on distinct streams are thread safe.
 *    If the workspace cannot be allocated, VQS_ENOMEM is returned and keys is
 *    untouched.
 *  - Sorting is not stable (Sec. 5): equal keys are bit-identical here, so the
 *    output is the unique sorted rearrangement of the input.
 */
#ifndef VQS_H
#define VQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types. */
enum vqs_key_type {
    VQS_U16 = 1,
    VQS_U32 = 2,
    VQS_U64 = 3,
    VQS_U128 = 4,
    VQS_F32 = 5,
    VQS_F64 = 6
};

/* Return codes: 0 on success, negative on failure. */
enum vqs_status {
    VQS_OK = 0,
    VQS_EINVAL = -1,     /* bad argument (null pointer, misaligned keys, bad option) */
    VQS_ETYPE = -2,      /* unknown key type */
    VQS_ENOMEM = -3,     /* workspace allocation failed */
    VQS_EHIP = -4,       /* a HIP runtime call failed */
    VQS_EOFFSETS = -5,   /* offsets decrease (checked only with options.validate) */
    VQS_EINTERNAL = -6,  /* a device-side capacity check failed (see vqs_last_error_bits) */
    VQS_ESIZE = -7       /* input too large for the fixed scratch of vqs_sort_noalloc */
};

/* Method selector of vqs_options.method. */
enum vqs_method {
    VQS_METHOD_PLAIN = 0,    /* the paper's Quicksort */
    VQS_METHOD_LEARNED = 1   /* learned 256-bucket splitter first, then the plain method */
};

/* How the device-wide partition levels place a tile's output (vqs_options.level_mode).
 * Both give identical results and recursion counts.
 *  - LOOKBACK: each tile finds its offsets inside its range from the left counts of
 *    the range's earlier tiles (a decoupled look-back), and the partition is written
 *    contiguously.
 *  - RUNS: each tile partitions into its own interval, with no waiting.  A child range
 *    is then held as one run per tile of its parent.  The next level gathers it
 *    through a run table, and a range leaving for a single workgroup is first gathered
 *    into place by one copy pass.
 *  - AUTO: RUNS for one array of 8- or 16-byte keys.  LOOKBACK for 2- and 4-byte
 *    keys, whose one-key gathers cost more than the look-back saves, and for many
 *    ranges at once (segmented sorts, the learned splitter's buckets), whose short
 *    look-back chains cost less than run mode's copy pass. */
enum vqs_level_mode {
    VQS_LEVEL_AUTO = 0,
    VQS_LEVEL_LOOKBACK = 1,
    VQS_LEVEL_RUNS = 2
};

/* Options of the extended entry points.  Zero-initialise and set struct_size;
 * every zero field selects the default. */
typedef struct vqs_options {
    uint32_t struct_size;       /* sizeof(vqs_options) */
    uint32_t method;            /* enum vqs_method */
    uint64_t seed;              /* seed of the pivot sampler (Sec. 2.2); default 0 */
    int64_t depth_limit;        /* 0: 2*floor(log2 n)+4 per range; > 0: that limit;
                                   < 0: limit 0 (every range above the base case
                                   takes the bounded-time fallback) */
    uint32_t base_case;         /* NBaseCase in keys, 32..256; default 256 */
    uint32_t local_keys;        /* LDS local-sort capacity in keys; default: tuned */
    uint64_t solo_max;          /* ranges up to this many keys are finished by one
                                   workgroup; default: tuned */
    uint32_t use_graph;         /* segmented sort: capture the launch sequence once in a
                                   hipGraph and replay it on later calls with the same
                                   arguments */
    uint32_t validate;          /* check offsets for monotonicity (synchronises) */
    /* learned splitter (method VQS_METHOD_LEARNED, u64 keys) */
    uint32_t train_steps;       /* optimiser steps; default 100 */
    uint32_t batch;             /* training minibatch, at most 256; default 256 */
    float sample_fraction;      /* fraction of keys sampled; default 0.01 */
    float overflow_factor;      /* a bucket above overflow_factor * n/256 keys is left
                                   to the plain method; default 2.0 */
    float learning_rate;        /* Adam step size; default 0.003 */
    uint64_t model_seed;        /* seed of the model's initial weights; default 16 */
    uint64_t sample_seed;       /* seed of the 1 % chunk sample and of the minibatches;
                                   default 17 */
    uint32_t level_mode;        /* enum vqs_level_mode; default VQS_LEVEL_AUTO */
    uint32_t reserved[2];
} vqs_options;

/* Counters of the last call on a stream (copied with synchronisation).  The first
 * eight count the recursion exactly like the CPU oracle does. */
typedef struct vqs_stats {
    uint64_t partitions;        /* Partition calls (all ranges, all levels) */
    uint64_t keys_partitioned;  /* sum of partitioned range lengths */
    uint64_t degenerate;        /* partitions with an empty right side */
    uint64_t all_equal;         /* degenerate ranges holding one value */
    uint64_t basecases;         /* BaseCase calls */
    uint64_t fallbacks;         /* ranges past the depth limit */
    uint64_t fallback_keys;     /* keys in those ranges */
    uint64_t max_depth;         /* deepest partitioning recursion */
    uint64_t levels;            /* device-wide partition levels launched with work */
    uint64_t level_tiles;       /* tiles processed by the level kernels */
    uint64_t solo_items;        /* ranges finished by single workgroups */
    uint64_t lds_partitions;    /* partitions done inside LDS */
    /* learned splitter */
    uint64_t learned_buckets;   /* buckets produced (0 if the plain method ran) */
    uint64_t overflow_buckets;  /* buckets above the overflow bound */
    uint64_t max_bucket;        /* largest bucket */
    double train_loss;          /* final minibatch loss */
} vqs_stats;

/* Sort keys[0, n) in place on the default stream with default options. */
int vqs_sort(void* keys, uint64_t n, int key_type, int ascending);

/* Sort each segment [offsets[i], offsets[i+1]) of keys independently, for
 * i < nseg.  offsets is a device array of nseg + 1 non-decreasing int64 values;
 * empty segments are allowed. */
int vqs_sort_segmented(void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending);

/* Extended forms: options may be NULL (defaults); stream is a hipStream_t or NULL. */
int vqs_sort_ex(void* keys, uint64_t n, int key_type, int ascending, const vqs_options* options,
                void* stream);
int vqs_sort_segmented_ex(void* keys, const int64_t* offsets, uint64_t nseg, int key_type,
                          int ascending, const vqs_options* options, void* stream);

/* ---- allocation-free sort ----------------------------------------------------------
 * For callers that cannot allocate device memory: serving loops that must not call
 * hipMalloc between requests, and harnesses that forbid allocation.
 *
 * The same sort as vqs_sort_ex on one array with the plain method (same kernels, same
 * result and counters), except that every workspace buffer -- the n-key ping-pong
 * scratch, range lists, tile tables, counters, statistics -- is carved from a fixed
 * device array of VQS_NOALLOC_SCRATCH_BYTES bytes.  The library holds one such array
 * per device it runs on, from its load until the process exits.  The call makes no
 * hipMalloc, hipFree, hipHostMalloc or event creation; the caller passes the keys.
 *
 *  - Limit: n is accepted iff vqs_workspace_bytes(n, 1, key_type, options) <=
 *    VQS_NOALLOC_SCRATCH_BYTES (with default options on a 256-CU device up to about
 *    7.2e7 u16, 3.9e7 u32 or f32, 2.0e7 u64 or f64, 1.0e7 u128 keys); a larger n
 *    returns VQS_ESIZE and launches nothing.
 *  - options: as for vqs_sort_ex, but method must be VQS_METHOD_PLAIN and use_graph
 *    0 (VQS_EINVAL otherwise).
 *  - Sharing: every call on a device uses that device's one array, which keeps the
 *    last call's contents (each call clears what it reads with a kernel first).  Calls
 *    that overlap on one device -- on two streams, or from two threads without
 *    ordering -- race on the array and corrupt each other's results: issue them on one
 *    stream or order them with events.
 *  - Synchronisation: as vqs_sort_ex, the host waits for the stream once per batch of
 *    recursion levels to read an 8-byte level counter (into a pageable host word), so
 *    the call cannot be captured into a HIP graph.
 *  - vqs_get_stats and vqs_last_error_bits on the same stream report this call until
 *    a later call on that stream. */
#define VQS_NOALLOC_SCRATCH_BYTES (256ull << 20)
int vqs_sort_noalloc(void* keys, uint64_t n, int key_type, int ascending, const vqs_options* options,
                     void* stream);

/* Autotuner of the batched (segmented) sort.  Times the sort with every combination
 * of the run-time tunables -- solo_max (ranges up to this many keys are finished by
 * one workgroup each, longer ones are partitioned by the device-wide level kernel) in
 * {0 = the library's size rule, 2^14, 2^16, 2^18, 2^20}, local_keys (size of the
 * in-LDS sort) in {full buffer, half}, base_case in {256, 128} -- on a copy of the
 * segments (all of them when max_keys is 0, else the longest prefix with at most
 * max_keys keys, at least one segment), best of two timed runs after a warm-up each,
 * and writes the fastest combination into options->solo_max, local_keys and base_case
 * (the other fields are kept and used for the runs; method is plain).  keys and
 * offsets are device pointers as for vqs_sort_segmented; the caller's keys are not
 * modified.  Allocates the copy (hipMalloc, freed before return) and synchronises the
 * stream.  *best_ms (if not NULL) receives the best time.  Errors: VQS_EINVAL for
 * null pointers, nseg == 0 or a short options struct, VQS_EOFFSETS, VQS_ENOMEM,
 * VQS_EHIP.  A prefix represents the batch only when the segment order carries no
 * size trend, and the best solo_max depends on how many ranges run at once, so a
 * prefix may prefer a smaller one than the whole batch. */
int vqs_autotune_segmented(const void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending,
                           uint64_t max_keys, vqs_options* options, float* best_ms, void* stream);

/* Device bytes of the workspace a sort of n keys (in nseg segments) needs. */
uint64_t vqs_workspace_bytes(uint64_t n, uint64_t nseg, int key_type, const vqs_options* options);

/* Statistics of the last call issued on `stream`; waits for that call to finish. */
int vqs_get_stats(void* stream, vqs_stats* out);

/* Device error bits of the last call on `stream` (0 if none); waits for it. */
int vqs_last_error_bits(void* stream, uint32_t* out);

/* ---- learned splitter pieces (method VQS_METHOD_LEARNED runs all of them) --------
 * The model is a 1 -> 32 -> 32 -> 1 perceptron with clamp-to-[0,1] activations and
 * non-negative weight matrices: its parameter block is 1155 floats on the device,
 * w1[32] b1[32] W2[32][32] (row j = second-layer unit j) b2[32] w3[32] b3 x0 xs.
 * Input of a key k: x(k) = float(bits(float(k))) * 2^-31; xn = (x - x0) * xs;
 * bucket(k) = min(255, floor(256 * y)).  All pointers are device pointers. */

/* Sample sample_fraction of the u64 keys in random 64-byte chunks, sort the sample,
 * compute mid-rank CDF targets and train (train_steps Adam steps, 0 meaning the
 * default; vqs_mlp_init gives the untrained model).  Writes the parameter block to
 * params (1155 floats). */
int vqs_learned_fit(const void* keys, uint64_t n, const vqs_options* options, float* params, void* stream);

/* y = model(x) for m inputs. */
int vqs_mlp_forward(const float* params, const float* x, uint64_t m, float* y, void* stream);

/* Gradient (1153 floats) and mean squared error of the model on m <= 256 samples
 * (x, target t). */
int vqs_mlp_gradient(const float* params, const float* x, const float* t, uint32_t m, float* grad, float* loss,
                     void* stream);

/* steps Adam steps on minibatches of `batch` <= 256 samples (random, from sample_seed,
 * or consecutive when sequential != 0).  moments holds 2*1153+1 floats (first and
 * second moments, zero to start; the last receives the final minibatch loss). */
int vqs_mlp_train(float* params, float* moments, const float* x, const float* t, uint64_t m, uint32_t steps,
                  uint32_t batch, float learning_rate, uint64_t sample_seed, int sequential, void* stream);

/* Initial (untrained) parameters for inputs x[0..m) sorted ascending. */
int vqs_mlp_init(float* params, uint64_t model_seed, const float* x, uint64_t m, void* stream);

/* bucket(k) by the model's forward pass, per key. */
int vqs_mlp_buckets(const float* params, const uint64_t* keys, uint64_t n, int32_t* out, void* stream);

/* The 255 exact thresholds t_j = min{k : bucket(k) >= j} (j = 1..255) and the number of
 * them that exist (bucket(2^64-1)); bucket(k) = #{j <= nvalid : t_j <= k}. */
int vqs_learned_thresholds(const float* params, uint64_t* thresholds, uint32_t* nvalid, void* stream);

/* bucket(k) by binary search over the thresholds, per key. */
int vqs_learned_classify(const uint64_t* keys, uint64_t n, const uint64_t* thresholds, const uint32_t* nvalid,
                         int32_t* out, void* stream);

/* Kernel timing records (profiling): one per kernel launch on a stream since the
 * records were last read, measured with HIP events recorded on that stream around
 * the launch. */
typedef struct vqs_kernel_time {
    int32_t kind;               /* 0 clear, 1 seed, 2 level partition, 3 solo, 4..7 learned,
                                   8 level pivots */
    int32_t level;              /* recursion level of a level launch, else -1 */
    uint64_t keys;              /* keys the launch partitions (level launches), else 0 */
    double ms;                  /* event-measured duration */
} vqs_kernel_time;

/* Event recording around the launches of later calls: 0 none, 1 every launch,
 * 2 only the device-wide partition launches (kind 2; the others run unrecorded, so
 * a timing of the whole call is barely disturbed).  Other values: VQS_EINVAL. */
int vqs_profile(int enable);

/* Copy up to max records of the calls on `stream` since the last read to out and
 * clear them; *count receives the number copied.  Waits for the stream. */
int vqs_profile_read(void* stream, vqs_kernel_time* out, int max, int* count);

/* Free every workspace held by the library (waits for pending work). */
int vqs_release(void);

/* Human-readable text of a return code. */
const char* vqs_strerror(int code);

/* Library version as major*10000 + minor*100 + patch. */
int vqs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VQS_H */
