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
 *  - Sorting is not stable (Sec. 5): equal keys are bit-identical here (for
 *    VQS_K64V64 equal keys are ordered by their data), so the output is the unique
 *    sorted rearrangement of the input.  vqs_sort_stable keeps equal keys in input
 *    order and returns the permutation.
 *  - Workspace: unless options.workspace supplies one, the library keeps a device
 *    workspace (a scratch array of n keys for the out-of-place partitions, none with
 *    options.inplace, plus range lists, tile tables and counters;
 *    vqs_workspace_bytes gives its size) per
 *    (device, stream), allocated on first use, grown when needed and reused.  If it
 *    cannot be allocated, VQS_ENOMEM is returned and keys is untouched.  Calls on
 *    distinct streams are thread safe.
 *  - Argument errors return at once without launching anything.  A failing HIP call
 *    returns VQS_EHIP.
 *
 * Synchronisation.  Work is issued on `stream` (a hipStream_t; NULL is the default
 * stream) and a call returns while its last kernels still run, except where the host
 * waits for the stream:
 *  - the level loop (vqs_sort, vqs_sort_ex, vqs_sort_noalloc, and the segmented
 *    forms without use_graph): when the input holds ranges longer than solo_max,
 *    the device-wide recursion levels are issued in batches (first
 *    floor(log2(n / solo_max)) + 6 levels, then 4 at a time) and after each batch
 *    the host waits for the stream and reads one 8-byte counter to see whether a
 *    level is left.  The per-workgroup finish (the last kernel) is in flight on
 *    return.  An input with no range longer than solo_max is issued without waiting;
 *  - segmented sorts read offsets[nseg] (the total key count) before issuing anything,
 *    unless options.total_keys supplies it; with options.validate every offset is read;
 *  - with options.use_graph, a segmented call replays one captured graph holding every
 *    level's launches, so with options.total_keys it does not wait at all (capture,
 *    on the first call with given arguments, does not wait either);
 *  - the learned method waits in the level loops of its sample's sort and of the
 *    buckets' sort;
 *  - vqs_autotune_segmented, vqs_get_stats, vqs_last_error_bits, vqs_profile_read and
 *    vqs_release wait for the stream (or all streams) before returning.
 */
#ifndef VQS_H
#define VQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types: the 16/32/64-bit integers, 32/64-bit floating point and pairs of 64-bit
 * halves forming a 128-bit key that the paper's method handles (Sec. 2.4, Sec. 5; its
 * measurements use signed i16/i32/i64 keys).  Every type sorts ascending or
 * descending (Sec. 2.4's order tag). */
enum vqs_key_type {
    VQS_U16 = 1,
    VQS_U32 = 2,
    VQS_U64 = 3,
    VQS_U128 = 4,
    VQS_F32 = 5,
    VQS_F64 = 6,
    VQS_I16 = 7,     /* two's-complement integers, signed order */
    VQS_I32 = 8,
    VQS_I64 = 9,
    VQS_K64V64 = 10  /* a 64-bit key with 64-bit associated data, 16 bytes: the data at
                        byte 0, the key at byte 8.  Sorted as the 128-bit key (key,
                        data), as Sec. 2.4 treats such pairs: keys in order, equal keys
                        ordered by their data, so the result is unique. */
};

/* Return codes: 0 on success, negative on failure. */
enum vqs_status {
    VQS_OK = 0,
    VQS_EINVAL = -1,     /* bad argument (null pointer, misaligned keys, bad option) */
    VQS_ETYPE = -2,      /* unknown key type */
    VQS_ENOMEM = -3,     /* workspace allocation failed */
    VQS_EHIP = -4,       /* a HIP runtime call failed */
    VQS_EOFFSETS = -5,   /* offsets decrease (checked only with options.validate), or
                            options.total_keys differs from offsets[nseg] (validate) */
    VQS_EINTERNAL = -6,  /* a device-side capacity check failed (see vqs_last_error_bits) */
    VQS_ESIZE = -7       /* input too large for the supplied workspace
                            (options.workspace_bytes) or for the fixed scratch of
                            vqs_sort_noalloc */
};

/* Method selector of vqs_options.method. */
enum vqs_method {
    VQS_METHOD_PLAIN = 0,    /* the paper's Quicksort (Alg. 1) */
    VQS_METHOD_LEARNED = 1   /* a 256-way split first, then the Quicksort on every bucket:
                                the samplesort-then-Quicksort hybrid of Sec. 4.2, with
                                the splitters given by a learned monotone CDF model */
};

/* How the device-wide partition levels place a tile's output (vqs_options.level_mode).
 * Both give identical results and recursion counts (the key sequence of Sec. 2.1's
 * partition is the same; only its placement in memory differs).
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
 * every zero field selects the default.  A field is read only when struct_size
 * covers it (struct_size 0 is taken as the full structure). */
typedef struct vqs_options {
    uint32_t struct_size;       /* sizeof(vqs_options) */
    uint32_t method;            /* enum vqs_method */
    uint64_t seed;              /* seed of the pivot sampler's generator (Sec. 2.2);
                                   default 0 */
    int64_t depth_limit;        /* recursion depth limit (Sec. 2.2): 0: 2*floor(log2 n)+4
                                   per range; > 0: that limit; < 0: limit 0 (every range
                                   above the base case takes the fallback) */
    uint32_t base_case;         /* NBaseCase in keys (Sec. 2.3), 32..256; default 256 */
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
    uint32_t fallback_limit;    /* depth limit of the fallback mode itself: a range past
                                   the paper's limit (Sec. 2.2) keeps being partitioned
                                   until this depth, then takes the bounded-time sort.
                                   0: 2*floor(log2 len)+4 of the range;
                                   VQS_FALLBACK_LIMIT_ZERO: 0, so such a range goes
                                   straight to the bounded-time sort */
    uint32_t tile_variant;      /* level partition tile size: 0 the default per key width
                                   (16 KB u16, 32 KB u32, 40 KB u64, 32 KB u128), 1 half
                                   of it (for batches of many short ranges); other values:
                                   VQS_EINVAL */
    uint64_t total_keys;        /* segmented sorts: offsets[nseg], if the caller knows it
                                   (then it is not read from the device); 0: read it */
    void* workspace;            /* optional caller-owned device workspace (256-byte
                                   aligned) used instead of the library's, so the call
                                   allocates no device memory.  Its contents are
                                   scratch; keep it until the call has finished and its
                                   statistics or error bits have been read.  Not with
                                   the learned method (VQS_EINVAL). */
    uint64_t workspace_bytes;   /* its size; below vqs_workspace_bytes(...): VQS_ESIZE */
    uint32_t rng;               /* pivot sampler's generator (Sec. 2.2): VQS_RNG_SFC64 (default,
                                   seeded by seed) or VQS_RNG_CHACHA20, the secure option:
                                   each range's nine chunk offsets come from one ChaCha20
                                   block (RFC 8439) under rng_key, with block counter = the
                                   low 32 bits of the range start b and nonce = (the high 32
                                   bits of b, the low and the high 32 bits of the range end),
                                   so sampling positions cannot be predicted without the
                                   key; other values: VQS_EINVAL */
    uint32_t rng_key[8];        /* the 256-bit ChaCha20 key as eight little-endian words */
    uint32_t reserved0;         /* zero */
    uint32_t inplace;           /* 1: partition in place, in the order of the paper's
                                   in-place bidirectional scan (Sec. 2.1: 64-key vectors,
                                   four per loop iteration; the side with less capacity
                                   is read next, the first and last blocks are held
                                   back), keeping no scratch array of keys: the
                                   workspace shrinks to about n / 40 keys of block
                                   counts and saved blocks plus the lists.  The result
                                   is the same sorted array; the recursion counters are
                                   those of the oracle's in-place Partition.  Plain
                                   method only, without use_graph or level_mode; other
                                   values: VQS_EINVAL */
} vqs_options;

/* Generators of vqs_options.rng. */
enum vqs_rng {
    VQS_RNG_SFC64 = 0,
    VQS_RNG_CHACHA20 = 1
};

#define VQS_FALLBACK_LIMIT_ZERO 0xFFFFFFFFu

/* Counters of the last call on a stream (copied with synchronisation).  The first
 * eight count the recursion of Alg. 1 exactly as the CPU oracle does: one Partition
 * per Recurse call that partitions, the degenerate re-partition with the first key
 * included; BaseCase calls; ranges past the depth limit (the oracle's HeapSort calls). */
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
    /* traffic and the bounded-time fallback */
    uint64_t hbm_read_keys;     /* keys read from device memory by whole-key sweeps: the
                                   level partitions and copy passes, the per-workgroup
                                   partitions, the load of every in-LDS sort, the
                                   bounded-time sorts' passes (partitions inside LDS,
                                   pivot samples, tile minima and the learned splitter's
                                   own passes are not counted) */
    uint64_t hbm_write_keys;    /* keys written by the same sweeps, fills included */
    uint64_t bounded_lds;       /* ranges sorted by the bounded-time network in LDS */
    uint64_t bounded_global;    /* ranges sorted by the bounded-time chunk sort and
                                   merge through device memory */
} vqs_stats;

/* Sort keys[0, n) in place, ascending (ascending = 1) or descending (0), on the
 * default stream with default options: Sec. 2.4's Sort(keys, n, order tag). */
int vqs_sort(void* keys, uint64_t n, int key_type, int ascending);

/* Sort each segment [offsets[i], offsets[i+1]) of keys independently, for
 * i < nseg, each as vqs_sort would (the same pivots, recursion and result per
 * segment), all in one sequence of launches.  offsets is a device array of nseg + 1
 * non-decreasing int64 values; empty segments are allowed.  Not in the paper: the
 * batched analogue of many independent Sort calls. */
int vqs_sort_segmented(void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending);

/* Extended forms of the two calls above: options may be NULL (defaults); stream is a
 * hipStream_t or NULL. */
int vqs_sort_ex(void* keys, uint64_t n, int key_type, int ascending, const vqs_options* options,
                void* stream);
int vqs_sort_segmented_ex(void* keys, const int64_t* offsets, uint64_t nseg, int key_type,
                          int ascending, const vqs_options* options, void* stream);

/* Stable sort (Sec. 5: Quicksort is not stable, but becomes so when a unique row
 * identifier is appended to the least-significant bits of each key).  Sorts keys[0, n)
 * in place so that equal keys keep their input order and, if rows is not NULL, writes
 * rows[i] = the input position of the key now at position i (device array of n
 * uint64, 8-byte aligned) -- the permutation to apply to any associated data.  Each
 * key's order-preserving unsigned form is joined with its row number into a
 * composite key, (key << 32) | row as a u64 for keys of up to 32 bits and n <= 2^32,
 * otherwise a 128-bit key (key, row); the composites (all distinct) are sorted by the
 * plain method and split again.  Key types of up to 64 bits (VQS_U128 and VQS_K64V64:
 * VQS_ETYPE).  options as for vqs_sort_ex, method plain, no caller workspace
 * (VQS_EINVAL otherwise); the composite array (n * 8 or n * 16 bytes) is a library
 * workspace per stream.  vqs_get_stats reports the composite sort.  Synchronisation as
 * vqs_sort_ex. */
int vqs_sort_stable(void* keys, uint64_t n, int key_type, int ascending, uint64_t* rows,
                    const vqs_options* options, void* stream);

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
 *    7.2e7 u16, 3.9e7 u32 or f32, 2.0e7 u64 or f64, 1.0e7 u128 keys; with
 *    options.inplace, which keeps no scratch array of keys, up to about 7.1e8 u16,
 *    6.6e8 u32, 5.8e8 u64, 2.5e8 u128 keys); a larger n returns VQS_ESIZE and
 *    launches nothing.
 *  - options: as for vqs_sort_ex, but method must be VQS_METHOD_PLAIN, use_graph 0
 *    and workspace NULL (VQS_EINVAL otherwise).
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
 * in-LDS sort) in {full buffer, half}, base_case in {256, 128}, level_mode in
 * {LOOKBACK, RUNS} and tile_variant (compiled level tile sizes) in {0, 1} -- on a copy
 * of the segments (all of them when max_keys is 0, else the longest prefix with at
 * most max_keys keys, at least one segment), best of two timed runs after a warm-up
 * each, and writes the fastest combination into options->solo_max, local_keys,
 * base_case, level_mode and tile_variant (the other fields are kept
 * and used for the runs; method is plain).  keys and offsets are device pointers as
 * for vqs_sort_segmented; the caller's keys are not modified.  Allocates the copy
 * (hipMalloc, freed before return) and synchronises the stream.  *best_ms (if not
 * NULL) receives the best time.  Errors: VQS_EINVAL for null pointers, nseg == 0 or a
 * short options struct, VQS_EOFFSETS, VQS_ENOMEM, VQS_EHIP.  A prefix represents the
 * batch only when the segment order carries no size trend, and the best solo_max
 * depends on how many ranges run at once, so a prefix may prefer a smaller one than
 * the whole batch.  Not in the paper. */
int vqs_autotune_segmented(const void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending,
                           uint64_t max_keys, vqs_options* options, float* best_ms, void* stream);

/* Device bytes of the workspace a plain sort of n keys in nseg segments (nseg 0 is
 * taken as 1) needs with these options (NULL: defaults) on the current device: the
 * size options.workspace must have, and the measure of vqs_sort_noalloc's limit.
 * 0 for an unknown key type or rejected options. */
uint64_t vqs_workspace_bytes(uint64_t n, uint64_t nseg, int key_type, const vqs_options* options);

/* Statistics of the last call issued on `stream` (the counters above); waits for
 * that call to finish.  All zero if no call has run on the stream. */
int vqs_get_stats(void* stream, vqs_stats* out);

/* Device error bits of the last call on `stream` (0 if none); waits for it. */
int vqs_last_error_bits(void* stream, uint32_t* out);

/* ---- learned splitter pieces (method VQS_METHOD_LEARNED runs all of them) --------
 * Not in the paper, which names the 256-way samplesort split as the bandwidth-friendly
 * generalisation of the partition (Sec. 4.2); here its splitters come from a CDF model.
 * The model is a 1 -> 32 -> 32 -> 1 perceptron with clamp-to-[0,1] activations and
 * non-negative weight matrices: its parameter block is 1155 floats on the device,
 * w1[32] b1[32] W2[32][32] (row j = second-layer unit j) b2[32] w3[32] b3 x0 xs.
 * Input of a key k: x(k) = float(bits(float(k))) * 2^-31; xn = (x - x0) * xs;
 * bucket(k) = min(255, floor(256 * y)).  All pointers are device pointers. */

/* Sample sample_fraction of the u64 keys in random 64-byte chunks (the unit of
 * Sec. 2.2's pivot sampling), sort the sample, compute mid-rank CDF targets and train
 * (train_steps Adam steps, 0 meaning the default; vqs_mlp_init gives the untrained
 * model).  Writes the parameter block to params (1155 floats). */
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
 * a timing of the whole call is barely disturbed).  Other values: VQS_EINVAL.
 * Calls through vqs_sort_noalloc record nothing. */
int vqs_profile(int enable);

/* Copy up to max records of the calls on `stream` since the last read to out and
 * clear them; *count receives the number copied.  Waits for the stream. */
int vqs_profile_read(void* stream, vqs_kernel_time* out, int max, int* count);

/* Free every workspace held by the library (waits for pending work).  The fixed
 * scratch of vqs_sort_noalloc is not freed. */
int vqs_release(void);

/* Human-readable text of a return code. */
const char* vqs_strerror(int code);

/* Library version as major*10000 + minor*100 + patch. */
int vqs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VQS_H */
