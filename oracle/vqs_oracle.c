/*
 * vqs_oracle.c -- plain, slow, scalar CPU oracle for the vectorized Quicksort of
 * Blacher, Giesen, Sanders and Wassenberg, "Vectorized and performance-portable
 * Quicksort" (2022).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg
 * of bench.py may load this library.  It shares no code, header or table with the
 * GPU library; the product path never calls it.
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -o liboracle.so vqs_oracle.c -lm
 *
 * What it computes:
 *  - vqo_sort / vqo_sort_segmented: the paper's Quicksort (Alg. 1 with Sec. 2.1-2.4),
 *    run scalar.  Its output is the unique sorted rearrangement of the input
 *    (equal keys are bit-identical because inputs exclude NaN and -0.0).
 *  - the pieces on their own, for parity tests of the GPU kernels: ChoosePivot,
 *    Partition, ScanMinMax, BaseCase, Heapsort, the random generator and the
 *    networks as comparator lists.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - random bits: standard SFC64; per range its state comes from SplitMix64 over
 *    (seed, begin, end), so a range's pivot is a pure function of its contents and
 *    position; five 64-bit draws give ten 32-bit values, low half first, the first
 *    nine of which map to chunk offsets by the multiply-shift (Lemire) reduction.
 *  - Partition keeps left keys in input order and right keys in reverse input order
 *    (the paper's in-place scan leaves the order within a side unspecified).
 *  - the depth of the first Recurse call is 1; a call deeper than 2*floor(log2 n)+4
 *    Heapsorts its range; the degenerate re-partition counts as a recursion.
 *  - degenerate pivot: the first key in sort order (minimum ascending, maximum
 *    descending); padding: the last value in sort order.
 *  - key types: unsigned 16/32/64/128-bit, float, double (Sec. 2.4), and the signed
 *    16/32/64-bit integers of the paper's measurements; a 64-bit key with 64-bit
 *    associated data is a 128-bit key with the key in the upper half (Sec. 2.4), so
 *    equal keys are ordered by their data and the result stays unique.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VQO_U16 1
#define VQO_U32 2
#define VQO_U64 3
#define VQO_U128 4
#define VQO_F32 5
#define VQO_F64 6
#define VQO_I16 7
#define VQO_I32 8
#define VQO_I64 9
#define VQO_K64V64 10   /* 64-bit key in the upper half, 64-bit value in the lower: a 128-bit key */

typedef struct {
    uint64_t partitions;        /* Partition calls */
    uint64_t keys_partitioned;  /* sum of range lengths over Partition calls */
    uint64_t degenerate;        /* partitions whose right side was empty */
    uint64_t all_equal;         /* degenerate ranges found to hold one value */
    uint64_t basecases;         /* BaseCase calls on non-empty ranges */
    uint64_t heapsorts;         /* depth-limit fallbacks */
    uint64_t heapsort_keys;     /* keys sorted by the fallback */
    uint64_t max_depth;         /* deepest Recurse call that partitioned */
    uint64_t depth_limit_used;  /* limit applied to the last range sorted */
} vqo_stats;

typedef struct {
    int ascending;
    uint64_t seed;
    uint64_t nb;           /* NBaseCase: ranges of at most nb keys go to BaseCase */
    int64_t depth_limit;   /* < 0: 2*floor(log2 n)+4 */
    int rng;               /* 0: SFC64 from the seed; 1: ChaCha20 under key (the secure option) */
    uint32_t key[8];
    int inplace;           /* 1: the in-place bidirectional Partition of Sec. 2.1 */
} vqo_params;

/* ---- random numbers (Sec. 2.2) ---------------------------------------------- */

/* SplitMix64 (Steele, Lea, Flood 2014): add the golden-ratio increment, then the
 * variant-13 finalizer. */
uint64_t vqo_splitmix64_next(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* SFC64 (Doty-Humphrey's small fast chaotic generator), state {a, b, c, counter}. */
static uint64_t sfc64_next(uint64_t s[4]) {
    const uint64_t out = s[0] + s[1] + s[3];
    s[3] += 1;
    s[0] = s[1] ^ (s[1] >> 11);
    s[1] = s[2] + (s[2] << 3);
    s[2] = ((s[2] << 24) | (s[2] >> 40)) + out;
    return out;
}

void vqo_sfc64_raw(uint64_t state[4], uint64_t* out, uint64_t count) {
    for (uint64_t i = 0; i < count; i++) out[i] = sfc64_next(state);
}

/* State of the sampler for the range [b, e): SplitMix64 started at seed, with b and
 * then e mixed into its state before the draws that become a, b and c; counter 1;
 * then twelve outputs are discarded, as in SFC64's customary seeding. */
static void seg_rng_state(uint64_t seed, uint64_t b, uint64_t e, uint64_t s[4]) {
    uint64_t x = seed;
    x ^= b;
    s[0] = vqo_splitmix64_next(&x);
    x ^= e;
    s[1] = vqo_splitmix64_next(&x);
    s[2] = vqo_splitmix64_next(&x);
    s[3] = 1;
    for (int i = 0; i < 12; i++) (void)sfc64_next(s);
}

void vqo_seg_rng_state(uint64_t seed, uint64_t b, uint64_t e, uint64_t out[4]) {
    seg_rng_state(seed, b, e, out);
}

/* Division-free reduction of a 32-bit draw to [0, range): (u * range) >> 32.  One
 * draw per value; value v is hit by ceil or floor of 2^32/range draws, so the bias
 * is below range / 2^32.  Requires range < 2^32. */
static uint64_t multiply_shift_offset(uint32_t u, uint64_t range) {
    return ((uint64_t)u * range) >> 32;
}

uint64_t vqo_multiply_shift(uint32_t u, uint64_t range) { return multiply_shift_offset(u, range); }

/* ChaCha20 (Bernstein; the block function as specified in RFC 8439, Sec. 2.3): a
 * 4x4 state of 32-bit words -- the constants "expand 32-byte k", the 256-bit key, a
 * 32-bit block counter, a 96-bit nonce -- run through 20 rounds (10 column rounds
 * and 10 diagonal rounds of the quarter round), then added to the initial state. */
static uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

static void quarter_round(uint32_t* a, uint32_t* b, uint32_t* c, uint32_t* d) {
    *a += *b; *d ^= *a; *d = rotl32(*d, 16);
    *c += *d; *b ^= *c; *b = rotl32(*b, 12);
    *a += *b; *d ^= *a; *d = rotl32(*d, 8);
    *c += *d; *b ^= *c; *b = rotl32(*b, 7);
}

void vqo_chacha20_quarter_round(uint32_t v[4]) { quarter_round(&v[0], &v[1], &v[2], &v[3]); }

void vqo_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]) {
    uint32_t x[16];
    x[0] = 0x61707865u; x[1] = 0x3320646eu; x[2] = 0x79622d32u; x[3] = 0x6b206574u;
    for (int i = 0; i < 8; i++) x[4 + i] = key[i];
    x[12] = counter;
    x[13] = nonce[0]; x[14] = nonce[1]; x[15] = nonce[2];
    uint32_t w[16];
    memcpy(w, x, sizeof(w));
    for (int r = 0; r < 10; r++) {
        quarter_round(&w[0], &w[4], &w[8], &w[12]);
        quarter_round(&w[1], &w[5], &w[9], &w[13]);
        quarter_round(&w[2], &w[6], &w[10], &w[14]);
        quarter_round(&w[3], &w[7], &w[11], &w[15]);
        quarter_round(&w[0], &w[5], &w[10], &w[15]);
        quarter_round(&w[1], &w[6], &w[11], &w[12]);
        quarter_round(&w[2], &w[7], &w[8], &w[13]);
        quarter_round(&w[3], &w[4], &w[9], &w[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = w[i] + x[i];
}

/* The ten 32-bit random values of the range [b, e).  SFC64 (default): the five 64-bit
 * draws of the range's generator, low half first.  ChaCha20 (Sec. 2.2's secure
 * generator, which the paper builds from AES rounds): the first ten words of the
 * block with the caller's key, block counter = the low 32 bits of b, nonce = (the high
 * 32 bits of b, the low and the high 32 bits of e), so each range draws from its own
 * block and the draws stay a pure function of (key, b, e). */
static void range_draws(const vqo_params* p, uint64_t b, uint64_t e, uint32_t u[10]) {
    if (p->rng == 1) {
        uint32_t blk[16];
        const uint32_t nonce[3] = {(uint32_t)(b >> 32), (uint32_t)e, (uint32_t)(e >> 32)};
        vqo_chacha20_block(p->key, (uint32_t)b, nonce, blk);
        for (int i = 0; i < 10; i++) u[i] = blk[i];
        return;
    }
    uint64_t st[4];
    seg_rng_state(p->seed, b, e, st);
    for (int i = 0; i < 5; i++) {
        uint64_t r = sfc64_next(st);
        u[2 * i] = (uint32_t)r;
        u[2 * i + 1] = (uint32_t)(r >> 32);
    }
}

/* The nine chunk offsets (in chunks) ChoosePivot uses for [b, e) with w keys per
 * chunk; rng 0 draws from SFC64 seeded by seed, rng 1 from ChaCha20 under key. */
void vqo_pivot_offsets_rng(uint64_t seed, int rng, const uint32_t key[8], uint64_t b, uint64_t e, uint64_t w,
                           uint64_t out[9]) {
    vqo_params p;
    memset(&p, 0, sizeof(p));
    p.seed = seed;
    p.rng = rng;
    if (key) memcpy(p.key, key, sizeof(p.key));
    uint32_t u[10];
    range_draws(&p, b, e, u);
    for (int i = 0; i < 9; i++) out[i] = multiply_shift_offset(u[i], (e - b) / w);
}

void vqo_pivot_offsets(uint64_t seed, uint64_t b, uint64_t e, uint64_t w, uint64_t out[9]) {
    vqo_pivot_offsets_rng(seed, 0, NULL, b, e, w, out);
}

static uint64_t default_depth_limit(uint64_t n) {
    uint64_t lg = 0;
    while ((n >> (lg + 1)) != 0) lg++;              /* floor(log2 n) */
    return 2 * lg + 4;
}

uint64_t vqo_default_depth_limit(uint64_t n) { return default_depth_limit(n); }

/* ---- networks (Sec. 3) ------------------------------------------------------- */

/* Green's 16-input network (Knuth, TAOCP vol. 3, Sec. 5.3.4): four hypercube
 * layers, then 28 modules; 60 compare-and-exchange modules, 10 layers. */
#define GREEN16_MODULES 60
static const uint32_t GREEN16[GREEN16_MODULES][2] = {
    {0, 1}, {2, 3}, {4, 5}, {6, 7}, {8, 9}, {10, 11}, {12, 13}, {14, 15},
    {0, 2}, {1, 3}, {4, 6}, {5, 7}, {8, 10}, {9, 11}, {12, 14}, {13, 15},
    {0, 4}, {1, 5}, {2, 6}, {3, 7}, {8, 12}, {9, 13}, {10, 14}, {11, 15},
    {0, 8}, {1, 9}, {2, 10}, {3, 11}, {4, 12}, {5, 13}, {6, 14}, {7, 15},
    {5, 10}, {6, 9}, {3, 12}, {13, 14}, {7, 11}, {1, 2}, {4, 8},
    {1, 4}, {7, 13}, {2, 8}, {11, 14}, {5, 6}, {9, 10},
    {2, 4}, {11, 13}, {3, 8}, {7, 12},
    {6, 8}, {10, 12}, {3, 5}, {7, 9},
    {3, 4}, {5, 6}, {7, 8}, {9, 10}, {11, 12},
    {6, 7}, {8, 9},
};

int vqo_green16(uint32_t* out_pairs) {
    for (int m = 0; m < GREEN16_MODULES; m++) {
        out_pairs[2 * m] = GREEN16[m][0];
        out_pairs[2 * m + 1] = GREEN16[m][1];
    }
    return GREEN16_MODULES;
}

/* Bitonic merge network for two sorted halves of a sequence of length len (a power
 * of two): the flip stage compares i with len-1-i, then half-cleaners compare i with
 * i+d for d = len/4, ..., 1 (bit d of i clear).  For len = 8 this is exactly the
 * paper's Fig. 2 example (1,8)(2,7)(3,6)(4,5); (1,3)(2,4)(5,7)(6,8); adjacent pairs.
 * Built once per length and cached. */
#define MAX_MERGE_LOG2 16
static uint32_t (*merge_cache[MAX_MERGE_LOG2 + 1])[2];
static int merge_cache_n[MAX_MERGE_LOG2 + 1];

static const uint32_t (*merge_network(uint64_t len, int* npairs))[2] {
    int lg = 0;
    while ((1ull << lg) < len) lg++;
    if (!merge_cache[lg]) {
        const uint64_t half = len / 2;
        int stages = lg;                            /* flip + (lg - 1) half-cleaners */
        uint32_t(*net)[2] = malloc(sizeof(*net) * half * (uint64_t)stages);
        int m = 0;
        for (uint64_t i = 0; i < half; i++) {
            net[m][0] = (uint32_t)i;
            net[m][1] = (uint32_t)(len - 1 - i);
            m++;
        }
        for (uint64_t d = half / 2; d >= 1; d /= 2)
            for (uint64_t i = 0; i < len; i++)
                if ((i & d) == 0) {
                    net[m][0] = (uint32_t)i;
                    net[m][1] = (uint32_t)(i + d);
                    m++;
                }
        merge_cache_n[lg] = m;
        merge_cache[lg] = net;
    }
    *npairs = merge_cache_n[lg];
    return (const uint32_t(*)[2])merge_cache[lg];
}

int vqo_merge_network(uint64_t len, uint32_t* out_pairs) {
    int n = 0;
    const uint32_t(*net)[2] = merge_network(len, &n);
    for (int m = 0; m < n; m++) {
        out_pairs[2 * m] = net[m][0];
        out_pairs[2 * m + 1] = net[m][1];
    }
    return n;
}

/* The whole BaseCase network for 16*c cells (Sec. 2.3, Sec. 3), as one list of
 * compare-and-exchange modules on the cells of the row-major 16 x c matrix: Green's
 * 60 modules down each of the c columns, then for w = 1, 2, ... < c the bitonic merge
 * of every pair of adjacent sorted w-column groups, applied to each group's elements
 * in row-major order.  A merge reads its group's row-major sequence from the cells
 * where the previous stage left it (where[q] is the cell holding matrix position q),
 * so no data moves between stages; afterwards order[k] = where[k] is the cell holding
 * the k-th key in sort order.  The same list drives the base case below and the 0-1
 * checker of the tests.  Built for c = 1, 2, ..., 64 when the library loads. */
#define BC_LOG2_MAX_C 6
#define BC_MAX_CELLS (16u << BC_LOG2_MAX_C)
#define BC_MAX_MODULES 32768
typedef struct {
    int nmod;
    uint32_t cells;
    uint32_t pairs[BC_MAX_MODULES][2];
    uint32_t order[BC_MAX_CELLS];
} bc_net;
static bc_net BC_NET[BC_LOG2_MAX_C + 1];

static void build_basecase_network(uint64_t c, bc_net* out) {
    static uint32_t where[BC_MAX_CELLS], nw[BC_MAX_CELLS];
    const uint64_t cells = 16 * c;
    int m = 0;
    for (uint64_t q = 0; q < cells; q++) where[q] = (uint32_t)q;
    for (uint64_t j = 0; j < c; j++)
        for (int g = 0; g < GREEN16_MODULES; g++) {
            out->pairs[m][0] = (uint32_t)(GREEN16[g][0] * c + j);
            out->pairs[m][1] = (uint32_t)(GREEN16[g][1] * c + j);
            m++;
        }
    for (uint64_t w = 1; w < c; w *= 2) {
        const uint64_t L = 16 * w;                 /* keys per input group */
        int npairs = 0;
        const uint32_t(*net)[2] = merge_network(2 * L, &npairs);
        memcpy(nw, where, sizeof(uint32_t) * cells);
        for (uint64_t g0 = 0; g0 < c; g0 += 2 * w) {
            uint32_t in[BC_MAX_CELLS];             /* matrix position of sequence element k */
            for (uint64_t k = 0; k < L; k++) {
                in[k] = (uint32_t)((k / w) * c + g0 + k % w);
                in[L + k] = (uint32_t)((k / w) * c + g0 + w + k % w);
            }
            for (int t = 0; t < npairs; t++) {
                out->pairs[m][0] = where[in[net[t][0]]];
                out->pairs[m][1] = where[in[net[t][1]]];
                m++;
            }
            for (uint64_t k = 0; k < 2 * L; k++) nw[(k / (2 * w)) * c + g0 + k % (2 * w)] = where[in[k]];
        }
        memcpy(where, nw, sizeof(uint32_t) * cells);
    }
    out->nmod = m;
    out->cells = (uint32_t)cells;
    memcpy(out->order, where, sizeof(uint32_t) * cells);
}

__attribute__((constructor)) static void build_networks(void) {
    for (int lc = 0; lc <= BC_LOG2_MAX_C; lc++) build_basecase_network(1ull << lc, &BC_NET[lc]);
}

/* The network BaseCase applies to n keys (c the smallest power of two with 16c >= n):
 * modules to pairs (2 per module), the output order to order, the cell count to
 * *cells; returns the number of modules, or -1 for n > 1024. */
int vqo_basecase_network(uint64_t n, uint32_t* pairs, uint32_t* order, uint32_t* cells) {
    int lc = 0;
    while ((16ull << lc) < n) lc++;
    if (lc > BC_LOG2_MAX_C) return -1;
    const bc_net* net = &BC_NET[lc];
    for (int m = 0; m < net->nmod; m++) {
        pairs[2 * m] = net->pairs[m][0];
        pairs[2 * m + 1] = net->pairs[m][1];
    }
    memcpy(order, net->order, sizeof(uint32_t) * net->cells);
    *cells = net->cells;
    return net->nmod;
}

/* ---- per-type instantiation ---------------------------------------------------- */

#define CAT2(a, b) a##_##b
#define CAT(a, b) CAT2(a, b)

#define KT uint16_t
#define SFX(n) CAT(n, u16)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((uint16_t)0xFFFF)
#define KMINV ((uint16_t)0)
#define KW 32
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT uint32_t
#define SFX(n) CAT(n, u32)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((uint32_t)0xFFFFFFFFu)
#define KMINV ((uint32_t)0)
#define KW 16
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT uint64_t
#define SFX(n) CAT(n, u64)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((uint64_t)0xFFFFFFFFFFFFFFFFull)
#define KMINV ((uint64_t)0)
#define KW 8
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

/* 128-bit keys (Sec. 2.4): little-endian, low 64-bit word first in memory, so the
 * compiler's unsigned __int128 compares exactly as Alg. 2 (upper half first). */
typedef unsigned __int128 u128_t;
#define KT u128_t
#define SFX(n) CAT(n, u128)
#define KLESS(a, b) ((a) < (b))
#define KMAXV (~(u128_t)0)
#define KMINV ((u128_t)0)
#define KW 4
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT float
#define SFX(n) CAT(n, f32)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((float)INFINITY)
#define KMINV ((float)-INFINITY)
#define KW 16
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT double
#define SFX(n) CAT(n, f64)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((double)INFINITY)
#define KMINV ((double)-INFINITY)
#define KW 8
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

/* Signed integers (the i16 / i32 / i64 keys of the paper's measurements): the
 * natural signed order. */
#define KT int16_t
#define SFX(n) CAT(n, i16)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((int16_t)INT16_MAX)
#define KMINV ((int16_t)INT16_MIN)
#define KW 32
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT int32_t
#define SFX(n) CAT(n, i32)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((int32_t)INT32_MAX)
#define KMINV ((int32_t)INT32_MIN)
#define KW 16
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

#define KT int64_t
#define SFX(n) CAT(n, i64)
#define KLESS(a, b) ((a) < (b))
#define KMAXV ((int64_t)INT64_MAX)
#define KMINV ((int64_t)INT64_MIN)
#define KW 8
#include "oracle_body.h"
#undef KT
#undef SFX
#undef KLESS
#undef KMAXV
#undef KMINV
#undef KW

/* ---- exported API ---------------------------------------------------------------- */

static int key_size(int kt) {
    switch (kt) {
        case VQO_U16: case VQO_I16: return 2;
        case VQO_U32: case VQO_F32: case VQO_I32: return 4;
        case VQO_U64: case VQO_F64: case VQO_I64: return 8;
        case VQO_U128: case VQO_K64V64: return 16;
        default: return 0;
    }
}

int vqo_key_size(int kt) { return key_size(kt); }

#define DISPATCH(kt, call)                                   \
    switch (kt) {                                            \
        case VQO_U16: { call(u16, uint16_t); break; }        \
        case VQO_U32: { call(u32, uint32_t); break; }        \
        case VQO_U64: { call(u64, uint64_t); break; }        \
        case VQO_U128: { call(u128, u128_t); break; }        \
        case VQO_K64V64: { call(u128, u128_t); break; }      \
        case VQO_F32: { call(f32, float); break; }           \
        case VQO_F64: { call(f64, double); break; }          \
        case VQO_I16: { call(i16, int16_t); break; }         \
        case VQO_I32: { call(i32, int32_t); break; }         \
        case VQO_I64: { call(i64, int64_t); break; }         \
        default: return -2;                                  \
    }

/* Sort each segment [offsets[i], offsets[i+1]) of keys independently; a plain sort
 * is one segment.  nb must be at least 32 (so every partitioned range holds a whole
 * sampling chunk) and depth_limit < 0 selects the paper's limit.  Stats accumulate
 * over all segments.  Returns 0, or a negative error. */
int vqo_sort_segmented_opts(void* keys, const int64_t* offsets, uint64_t nseg, int kt, int ascending,
                            uint64_t seed, int rng, const uint32_t key[8], uint64_t nb, int64_t depth_limit,
                            int inplace, vqo_stats* st) {
    if (nb < 32) return -1;
    if (rng != 0 && rng != 1) return -1;
    if (inplace != 0 && inplace != 1) return -1;
    vqo_params p;
    memset(&p, 0, sizeof(p));
    p.ascending = ascending ? 1 : 0;
    p.seed = seed;
    p.nb = nb;
    p.depth_limit = depth_limit;
    p.rng = rng;
    p.inplace = inplace;
    if (key) memcpy(p.key, key, sizeof(p.key));
    vqo_stats local;
    memset(&local, 0, sizeof(local));
    uint64_t maxlen = 0;
    for (uint64_t i = 0; i < nseg; i++) {
        if (offsets[i + 1] < offsets[i] || offsets[i] < 0) return -5;
        uint64_t len = (uint64_t)(offsets[i + 1] - offsets[i]);
        if (len > maxlen) maxlen = len;
    }
    /* the out-of-place Partition's buffer; the in-place one needs none */
    void* tmp = malloc((size_t)(offsets[nseg] > 0 && !inplace ? offsets[nseg] : 1) * (size_t)key_size(kt));
    if (!tmp) return -3;
#define SORT_SEGS(sfx, T)                                                                     \
    for (uint64_t i = 0; i < nseg; i++)                                                       \
        sort_range_##sfx((T*)keys, (T*)tmp, (uint64_t)offsets[i], (uint64_t)offsets[i + 1], &p, \
                         &local);
    switch (kt) {
        case VQO_U16: SORT_SEGS(u16, uint16_t); break;
        case VQO_U32: SORT_SEGS(u32, uint32_t); break;
        case VQO_U64: SORT_SEGS(u64, uint64_t); break;
        case VQO_U128: case VQO_K64V64: SORT_SEGS(u128, u128_t); break;
        case VQO_F32: SORT_SEGS(f32, float); break;
        case VQO_F64: SORT_SEGS(f64, double); break;
        case VQO_I16: SORT_SEGS(i16, int16_t); break;
        case VQO_I32: SORT_SEGS(i32, int32_t); break;
        case VQO_I64: SORT_SEGS(i64, int64_t); break;
        default: free(tmp); return -2;
    }
#undef SORT_SEGS
    free(tmp);
    if (st) *st = local;
    return 0;
}

int vqo_sort_segmented_rng(void* keys, const int64_t* offsets, uint64_t nseg, int kt, int ascending,
                           uint64_t seed, int rng, const uint32_t key[8], uint64_t nb, int64_t depth_limit,
                           vqo_stats* st) {
    return vqo_sort_segmented_opts(keys, offsets, nseg, kt, ascending, seed, rng, key, nb, depth_limit, 0, st);
}

int vqo_sort_segmented(void* keys, const int64_t* offsets, uint64_t nseg, int kt, int ascending,
                       uint64_t seed, uint64_t nb, int64_t depth_limit, vqo_stats* st) {
    return vqo_sort_segmented_rng(keys, offsets, nseg, kt, ascending, seed, 0, NULL, nb, depth_limit, st);
}

int vqo_sort(void* keys, uint64_t n, int kt, int ascending, uint64_t seed, uint64_t nb,
             int64_t depth_limit, vqo_stats* st) {
    int64_t offs[2] = {0, (int64_t)n};
    return vqo_sort_segmented(keys, offs, 1, kt, ascending, seed, nb, depth_limit, st);
}

/* ChoosePivot for the range [b, e) of keys; writes the pivot key to *pivot_out. */
int vqo_choose_pivot_rng(const void* keys, uint64_t b, uint64_t e, int kt, int ascending, uint64_t seed,
                         int rng, const uint32_t key[8], void* pivot_out) {
    const int ks = key_size(kt);
    if (ks == 0) return -2;
    if ((e - b) < (uint64_t)(64 / ks)) return -1;   /* needs one whole chunk */
    vqo_params prm;
    memset(&prm, 0, sizeof(prm));
    prm.ascending = ascending ? 1 : 0;
    prm.seed = seed;
    prm.rng = rng;
    if (key) memcpy(prm.key, key, sizeof(prm.key));
#define PIV(sfx, T)                                                                 \
    {                                                                               \
        T p = choose_pivot_##sfx((const T*)keys, b, e, &prm);                       \
        memcpy(pivot_out, &p, sizeof(T));                                           \
    }
    DISPATCH(kt, PIV)
#undef PIV
    return 0;
}

int vqo_choose_pivot(const void* keys, uint64_t b, uint64_t e, int kt, int ascending, uint64_t seed,
                     void* pivot_out) {
    return vqo_choose_pivot_rng(keys, b, e, kt, ascending, seed, 0, NULL, pivot_out);
}

/* Partition [b, e) of keys about *pivot in place; returns the bound. */
int64_t vqo_partition(void* keys, uint64_t b, uint64_t e, int kt, int ascending, const void* pivot) {
    const int ks = key_size(kt);
    if (ks == 0) return -2;
    void* tmp = malloc((size_t)(e > 0 ? e : 1) * (size_t)ks);
    int64_t bound = -1;
#define PART(sfx, T)                                                                           \
    {                                                                                          \
        T p;                                                                                   \
        memcpy(&p, pivot, sizeof(T));                                                          \
        bound = (int64_t)partition_##sfx((T*)keys, (T*)tmp, b, e, p, ascending ? 1 : 0);       \
    }
    switch (kt) {
        case VQO_U16: PART(u16, uint16_t); break;
        case VQO_U32: PART(u32, uint32_t); break;
        case VQO_U64: PART(u64, uint64_t); break;
        case VQO_U128: case VQO_K64V64: PART(u128, u128_t); break;
        case VQO_F32: PART(f32, float); break;
        case VQO_F64: PART(f64, double); break;
        case VQO_I16: PART(i16, int16_t); break;
        case VQO_I32: PART(i32, int32_t); break;
        case VQO_I64: PART(i64, int64_t); break;
        default: break;
    }
#undef PART
    free(tmp);
    return bound;
}

/* In-place Partition (Sec. 2.1) of [b, e) of keys about *pivot; returns the bound. */
int64_t vqo_partition_inplace(void* keys, uint64_t b, uint64_t e, int kt, int ascending, const void* pivot) {
    int64_t bound = -1;
#define PIP(sfx, T)                                                                            \
    {                                                                                          \
        T p;                                                                                   \
        memcpy(&p, pivot, sizeof(T));                                                          \
        bound = (int64_t)partition_inplace_##sfx((T*)keys, b, e, p, ascending ? 1 : 0);        \
    }
    DISPATCH(kt, PIP)
#undef PIP
    return bound;
}

/* First and last key of [b, e) in sort order. */
int vqo_minmax(const void* keys, uint64_t b, uint64_t e, int kt, int ascending, void* first,
               void* last) {
    if (e <= b) return -1;
#define MM(sfx, T)                                                                  \
    {                                                                               \
        T f, l;                                                                     \
        minmax_##sfx((const T*)keys, b, e, ascending ? 1 : 0, &f, &l);              \
        memcpy(first, &f, sizeof(T));                                               \
        memcpy(last, &l, sizeof(T));                                                \
    }
    DISPATCH(kt, MM)
#undef MM
    return 0;
}

/* BaseCase on keys[0, n) (n up to 16*64). */
int vqo_basecase(void* keys, uint64_t n, int kt, int ascending) {
    if (n > 1024) return -1;
#define BC(sfx, T) basecase_##sfx((T*)keys, n, ascending ? 1 : 0);
    DISPATCH(kt, BC)
#undef BC
    return 0;
}

/* Heapsort keys[0, n). */
int vqo_heapsort(void* keys, uint64_t n, int kt, int ascending) {
#define HS(sfx, T) heapsort_##sfx((T*)keys, n, ascending ? 1 : 0);
    DISPATCH(kt, HS)
#undef HS
    return 0;
}

/* Median of three with the network of Sec. 2.2, on u64 keys (for pinning). */
uint64_t vqo_med3_u64(uint64_t a, uint64_t b, uint64_t c, int ascending) {
    return med3_u64(a, b, c, ascending ? 1 : 0);
}
