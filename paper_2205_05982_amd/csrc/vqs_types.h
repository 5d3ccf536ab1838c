// vqs_types.h -- structures and launch constants shared by the kernels and the host.
#pragma once
#include <stdint.h>

namespace vqs {

struct u128k {
  uint64_t lo, hi;
};

// transform mode bits of the caller's keys
constexpr int MODE_FLOAT = 1;
constexpr int MODE_DESC = 2;
constexpr int MODE_SIGNED = 4;   // two's-complement integers: the sign bit flipped

#ifndef VQS_LEVEL_P
#define VQS_LEVEL_P 256
#endif
constexpr int LEVEL_P = VQS_LEVEL_P;  // threads per level-kernel workgroup
constexpr int LEVEL_NW = LEVEL_P / 64;  // its waves
// 16-byte chunks per thread of a level tile, by key width (measured): 16 KB tiles for
// u16 (its keys take one register each), 36 KB for u32 (four workgroups per CU; 2.5e8
// f32 -4.3 % against 32 KB), 40 KB for u64 (three per CU; 44 and 48 KB slower), 32 KB
// for u128
constexpr int level_chunks(int bits) { return bits == 16 ? 4 : bits == 32 ? 9 : bits == 64 ? 10 : 8; }
// the second compiled tile size (vqs_options.tile_variant = 1): half the chunks, for
// batches of many short ranges whose last, partial tiles would otherwise dominate
constexpr int level_chunks_half(int bits) { return level_chunks(bits) / 2; }
#ifndef VQS_SOLO_P
#define VQS_SOLO_P 512
#endif
constexpr int SOLO_P = VQS_SOLO_P;  // threads per solo-kernel workgroup
#ifndef VQS_LOCAL_BYTES
#define VQS_LOCAL_BYTES 32768
#endif
constexpr int LOCAL_BYTES = VQS_LOCAL_BYTES;  // one LDS buffer of the local sort
// 16-byte chunks per thread of a solo-kernel tile: a tile fills one LDS buffer (half
// of it for u16, whose keys take one register each)
constexpr int solo_chunks(int bits) { return (bits == 16 ? LOCAL_BYTES / 32 : LOCAL_BYTES / 16) / SOLO_P; }
#ifndef VQS_LOCAL_LIST_CAP
#define VQS_LOCAL_LIST_CAP 64
#endif
constexpr int LOCAL_LIST_CAP = VQS_LOCAL_LIST_CAP;  // ranges per LDS recursion level

// In-place partitions (Sec. 2.1, the bidirectional scan): a vector is one wavefront's
// 64 keys, a loop iteration reads a block of four vectors
constexpr int IP_V = 64;
constexpr int IP_U = 4;
constexpr int IP_B = IP_V * IP_U;
constexpr uint32_t IP_STASH = 3 * IP_B;   // keys saved per range: the remainder, the two held-back blocks
// loop blocks per in-place level tile: 32 KB of keys, at most 32 blocks (a thread then
// holds at most 16 keys)
constexpr uint32_t ip_steps_of(int key_bytes) {
  return 32768u / (uint32_t)(IP_B * key_bytes) < 32u ? 32768u / (uint32_t)(IP_B * key_bytes) : 32u;
}
// loop blocks per chunk of one workgroup's in-place partition: at most 16, so that a
// thread holds at most eight keys in the solo kernel
constexpr uint32_t ip_chunk_steps(int key_bytes) {
  return 32768u / (uint32_t)(IP_B * key_bytes) < 16u ? 32768u / (uint32_t)(IP_B * key_bytes) : 16u;
}
// loop blocks (main-loop iterations) of a range of len >= 2 * IP_B keys
constexpr uint64_t ip_loop_blocks(uint64_t len) { return len / IP_B - 2; }
// tiles of an in-place level for a range of len >= 2 * IP_B keys
constexpr uint64_t ip_tiles_of(uint64_t len, uint32_t steps) {
  return ip_loop_blocks(len) ? (ip_loop_blocks(len) + steps - 1) / steps : 1;
}
// in-place mode: the solo kernel's ranges (its block tables hold 256 blocks)
constexpr uint64_t IP_SOLO_MIN = 4 * IP_B, IP_SOLO_MAX = 256 * IP_B;

// ---- shared structures -------------------------------------------------------------

enum : uint32_t {
  SEG_OVERRIDE = 1u,   // pivot given (degenerate re-partition with the first key)
  SEG_SCRATCH = 2u,    // data lives in the scratch buffer (else in the caller's array)
  SEG_RAW = 4u,        // data not yet transformed (caller's array, never touched)
  SEG_FALLBACK = 8u,   // past the paper's depth limit: fallback mode
  SEG_FILL = 16u,      // all keys equal: write pv to [b, e) of the caller's array
  SEG_PIVOT = 32u,     // pv holds the range's pivot (computed before the level's launch)
  SEG_STRICT = 64u,    // split into keys before the pivot and keys equal to it
  SEG_BOUNDED = 128u,  // past the fallback mode's own depth limit: bounded-time sort
  SEG_RUNS = 256u,     // keys held as runs of the previous level's tiles (run mode)
  SEG_RIGHT = 512u,    // with SEG_RUNS: the right parts of those tiles, in reverse tile order
  SEG_COPY = 1024u,    // level entry that only gathers the runs into [b, e) (then solo)
  SEG_MAXK = 2048u,    // mx holds the range's largest key (internal form)
  SEG_MINR = 4096u,    // the range is the right part of the range whose tiles were
                       // [rt_b, rt_b + rt_n) in the level that made it (else the left part)
  SEG_SKIP = 8192u,    // finished while planning its level: the level's tiles of it do nothing
};

struct Seg {
  uint64_t b, e;
  uint32_t depth, limit;
  uint32_t flags, pad;
  uint64_t pv_lo, pv_hi;  // override pivot or fill value (internal form)
  uint32_t rt_b, rt_n;    // the parent range's tiles in the previous level (its run table in run mode)
  uint64_t mx_lo, mx_hi;  // SEG_MAXK: the range's largest key (internal form)
};

// Run mode: a tile of a planned level: its range (index in the level's list) and the
// first run it reads (run-held ranges)
struct TileRef {
  uint32_t seg, frun;
};

// Run mode: what a level tile left behind in its interval of the destination
// (pos .. pos + nv: nl left keys in input order, then the right keys reversed), and
// where its two parts start inside the left child (lp) and the right child (rp).
struct TileRun {
  uint64_t lp, rp, pos;
  uint32_t nl, nv;
};

// In-place partitions: a range of an in-place level, as its prologue leaves it for the
// counting and partition launches (left counts of the remainder and of the two
// held-back blocks, and the smallest of their keys)
struct IpRange {
  uint32_t lrem, cfirst, clast, pad;
  uint64_t mn_lo, mn_hi;   // smallest of the remainder and held-back keys (internal form)
};

struct LevelCtr {
  unsigned long long packed;  // (segments << 40) | tiles
  unsigned long long keys;    // keys in the level's ranges
  unsigned int ticket;
  unsigned int ticket2;       // in-place levels: tickets of the partition launch
  unsigned long long pad2;
};

struct SoloCtr {
  unsigned long long count;
  unsigned long long ticket;
  unsigned long long big, small;   // the order of service: long ranges first (solo_order_kernel)
};

// Counters of the recursion, comparable one to one with the oracle's.
struct DevStats {
  unsigned long long partitions, keys_partitioned, degenerate, all_equal, basecases, fallbacks,
      fallback_keys, max_depth;
  unsigned long long level_tiles, solo_items, lds_partitions, global_solo_partitions;
  unsigned long long fallback_partitions;
  unsigned long long hbm_read_keys, hbm_write_keys;   // keys moved by whole-key sweeps
  unsigned long long bounded_lds, bounded_global;     // ranges sorted by the bounded-time sorts
};

enum : uint32_t {
  ERR_LEVEL_OVERFLOW = 1u,
  ERR_SOLO_OVERFLOW = 2u,
  ERR_SPIN = 4u,
  ERR_LOCAL_OVERFLOW = 8u,
  ERR_STACK = 16u,
  ERR_NO_PIVOT = 32u,
};

struct Params {
  void* keys;            // caller's array
  void* scratch;         // ping-pong buffer, same 16-byte alignment offset as keys
  uint64_t n_total;
  int off;               // keys before the first 16-byte boundary: (addr % 16) / size
  int mode;              // MODE_FLOAT | MODE_DESC transform of the caller's keys
  uint64_t seed;
  uint32_t rng_mode;     // pivot sampler: 0 SFC64 from seed, 1 ChaCha20 under rng_key
  uint32_t rng_key[8];
  uint32_t nb;           // NBaseCase (<= 256)
  uint32_t local_cap;    // keys per LDS local sort (<= LDS buffer capacity)
  uint64_t solo_max;     // ranges up to this length go to the solo kernel
  Seg* lvl_segs[2];
  unsigned long long* lvl_tbase[2];
  LevelCtr* lvl_ctr;
  unsigned long long* flags;  // look-back words, one per tile
  u128k* tilemin;        // per-tile minimum (internal form)
  u128k* tilermin;       // per tile of a level: its smallest right key
  Seg* solo;
  uint32_t* solo_order;  // the solo list's order of service (indices into solo)
  SoloCtr* solo_ctr;
  DevStats* stats;
  unsigned int* err;
  uint64_t cap_lvl, cap_tiles, cap_solo;
  int level;
  int max_levels;
  int64_t fixed_limit;   // < 0: 2*floor(log2 len)+4 per input range; else this limit
  int64_t fb_limit;      // fallback mode's own limit: < 0: 2*floor(log2 len)+4 of the range; else this
  int seed_level;        // level of the first partition (1: input ranges live in scratch)
  int run_mode;          // level partitions write tile-local runs (no look-back)
  TileRun* runs[2];      // run mode: per-tile table of the current and the previous level
  TileRef* tref;         // run mode: range and first run of each tile of the level being planned
  uint32_t* tnl;         // run mode: left count of each tile of the level just partitioned
  int inplace;           // partitions in place (no key scratch): the paper's bidirectional order
  uint32_t ip_steps;     // in-place level tiles: loop blocks per tile
  void* ip_stash;        // in-place levels: per range, its remainder and held-back blocks
  unsigned long long* ip_pfx;   // in-place levels: left-count prefix of every loop block
  IpRange* ip_rng;       // in-place levels: per range, what its prologue found
  uint32_t* ip_tseg;     // in-place levels: the range of every tile
};

constexpr uint64_t FILL_CHUNK = 1ull << 16;
constexpr uint64_t TILE_MASK40 = (1ull << 40) - 1;

}  // namespace vqs
