// vqs_kernels.h -- HIP kernels of the vectorized Quicksort for gfx950.
//
// The paper's recursion (Alg. 1) is run breadth-first across the whole GPU:
//
//  * level partitions: one launch per recursion level.  Every range longer than the
//    "solo" threshold is cut into 16-byte-aligned tiles; all tiles of all ranges of
//    the level are partitioned in one persistent launch (atomic tile tickets).  Each
//    tile classifies its keys against its range's pivot (ChoosePivot, Sec. 2.2),
//    ranks them with wave ballots and prefix counts, stages them in LDS in compacted
//    order (the compress-store of Sec. 2.1) and writes them coalesced.  Two
//    placements of the output:
//      - level_runs_kernel: each tile writes its own interval; a child range is then
//        held as one run per tile of its parent, and runs_plan_kernel (before the
//        next partition launch) plans the ranges and records the runs;
//      - level_kernel: a tile's offset inside its range comes from a decoupled
//        look-back over the left counts of the preceding tiles; the last tile of a
//        range plans the children (pivots by pivot_kernel before each launch).
//    Small children go to the solo list, large ones to the next level.
//  * solo_kernel: one persistent launch; each workgroup takes whole ranges from the
//    solo list and finishes them alone: partition passes through global memory while
//    the range is larger than the LDS capacity, then the local sort in LDS
//    (partitions by single waves down to NBaseCase keys, then the 16x16 sorting
//    network of Sec. 3 in registers: Green's 60-module column network in every lane,
//    then transposition-free bitonic merges across lanes).
//
// Partition layout (both kernels, global and LDS): keys not after the pivot are
// written from the range start in input order, the others from the range end
// backwards (reverse input order).  This is the layout of the oracle's scalar
// out-of-place split, so pivots, ranges and recursion depths agree at every level.
//
// In-place mode (vqs_inplace.h) keeps no key scratch: every partition, device-wide,
// per workgroup or in LDS, leaves the order of the paper's in-place bidirectional
// scan (the oracle's in-place Partition), again so that the recursion agrees.
#pragma once
#include "vqs_device.h"
#include "vqs_types.h"

#include <type_traits>

namespace vqs {

__device__ inline void set_err(const Params& p, uint32_t e) { atomicOr(p.err, e); }

template <class K>
__device__ inline void to_words(typename K::R r, uint64_t& lo, uint64_t& hi) {
  K::to_u64x2(r, lo, hi);
}

template <class K>
__device__ inline typename K::R wave_min(typename K::R v) {
  // minimum within each row of 16 lanes by DPP exchanges (lane ^ 1, ^ 2, ^ 7, ^ 15: each
  // pairs the halves of the group the previous steps reduced), then the four row
  // minima read from lanes 0, 16, 32, 48: no LDS round trip
  v = K::kmin(v, xor_lanes<1>(v));
  v = K::kmin(v, xor_lanes<2>(v));
  v = K::kmin(v, xor_lanes<7>(v));
  v = K::kmin(v, xor_lanes<15>(v));
  const typename K::R r0 = read_lane(v, 0), r1 = read_lane(v, 16), r2 = read_lane(v, 32), r3 = read_lane(v, 48);
  return K::kmin(K::kmin(r0, r1), K::kmin(r2, r3));
}

// number of 16-byte-aligned tiles of T keys that intersect [b, e)
__device__ inline uint64_t tiles_of(uint64_t b, uint64_t e, int off, uint64_t T) {
  return (e - 1 + off) / T - (b + off) / T + 1;
}

__device__ inline uint32_t depth_limit_of(uint64_t n) {
  uint32_t lg = 63 - __clzll(n | 1);
  return 2 * lg + 4;
}

// depth limit of the fallback mode itself for a range of len keys
__device__ inline uint32_t fb_limit_of(const Params& p, uint64_t len) {
  return p.fb_limit >= 0 ? (uint32_t)p.fb_limit : depth_limit_of(len);
}

// ---- tile partition (workgroup) -------------------------------------------------------

template <class K, int P, int I>
struct Tile {
  using R = typename K::R;
  using S = typename K::S;
  static constexpr int V = K::V;
  static constexpr int NW = P / WAVE;
  static constexpr int TC = P * I;      // chunks per tile
  static constexpr int T = TC * V;      // keys per tile

  struct Aux {
    uint32_t cnt[I][NW];
    R wmin[NW];
    R pivot;
  };

  // Load the tile's chunks; key (j, q) of this thread sits at v-index
  // (k*TC + j*P + tid)*V + q.  Only chunks holding a key of [vs, ve) are read: a
  // 16-byte aligned load touching a valid key never leaves its page.
  // SPLIT: a separate path for tiles wholly inside the range (most of them), which need
  // no clamping (the solo kernel keeps one path: its registers are at their bound)
  template <bool SPLIT = true>
  __device__ static void load(const S* base_aligned, uint64_t k, uint64_t vs, uint64_t ve, int tmode,
                              R (&key)[I][V]) {
    if (SPLIT && vs == k * (uint64_t)T && ve == vs + T) load_t<true>(base_aligned, k, vs, ve, tmode, key);
    else load_t<false>(base_aligned, k, vs, ve, tmode, key);
  }
  template <bool FULL>
  __device__ static void load_t(const S* base_aligned, uint64_t k, uint64_t vs, uint64_t ve, int tmode,
                                R (&key)[I][V]) {
    const int tid = threadIdx.x;
    // All chunk loads are issued, unconditionally, before any value is used, so they
    // are in flight together (a use or a branch between them makes each wait for its
    // predecessor).  A chunk with no key of [vs, ve) reads the nearest chunk that has
    // one instead (always a safe address); its values are never used.
    const uint64_t cmin = vs / V, cmax = (ve - 1) / V;
    uint4 raw[I];
#pragma unroll
    for (int j = 0; j < I; j++) {
      uint64_t c = k * TC + (uint64_t)j * P + tid;
      if (!FULL) c = c < cmin ? cmin : (c > cmax ? cmax : c);
      raw[j] = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(base_aligned) + c * 16);
    }
#pragma unroll
    for (int j = 0; j < I; j++) {
      R tmp[V];
      K::unpack(raw[j], tmp);
#pragma unroll
      for (int q = 0; q < V; q++) {
        S s;
        if constexpr (sizeof(S) == sizeof(R)) {
          s = tmp[q];
        } else {
          s = (S)tmp[q];
        }
        key[j][q] = tmode ? K::load_t(s, tmode) : tmp[q];
      }
    }
  }

  // Classify against the pivot (left: not after it; strict: before it), rank stably,
  // stage in LDS (left keys from 0 upward, right keys from nvalid-1 downward).  Returns
  // the tile's left count; *tmin gets the tile minimum (thread 0), and thread 0 calls
  // publish(left count, minimum) as soon as both are known, before the keys are
  // staged.  Ends with a barrier.
  template <class Pub>
  __device__ static uint32_t rank_and_stage(S* stage, Aux& sh, const R (&key)[I][V], uint64_t k,
                                            uint64_t vs, uint64_t ve, R pivot, bool strict, R* tmin,
                                            Pub&& publish) {
    // A path for tiles wholly inside the range (no bounds per key) only for 2-byte keys:
    // wider keys' kernels would need more than 168 registers with both paths inlined,
    // which leaves two waves per SIMD instead of three (measured slower).
    if constexpr (sizeof(S) == 2) {
      if (vs == k * (uint64_t)T && ve == vs + T)
        return strict ? rank_and_stage_t<true, true>(stage, sh, key, k, vs, ve, pivot, tmin, publish)
                      : rank_and_stage_t<false, true>(stage, sh, key, k, vs, ve, pivot, tmin, publish);
    }
    return strict ? rank_and_stage_t<true, false>(stage, sh, key, k, vs, ve, pivot, tmin, publish)
                  : rank_and_stage_t<false, false>(stage, sh, key, k, vs, ve, pivot, tmin, publish);
  }
  // ST: strict split; FULL: every key of the tile is in the range
  template <bool ST, bool FULL, class Pub>
  __device__ static uint32_t rank_and_stage_t(S* stage, Aux& sh, const R (&key)[I][V], uint64_t k,
                                              uint64_t vs, uint64_t ve, R pivot, R* tmin, Pub& publish) {
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    uint32_t pre[I];
    uint32_t flag[I];  // bit q: key (j, q) goes left
    R mn = K::maxv();
    // positions relative to the tile's first v-index, so that bounds take 32-bit compares
    const uint64_t tb = k * (uint64_t)T;
    const uint32_t rlo = (uint32_t)(vs - tb), rhi = (uint32_t)(ve - tb);
#pragma unroll
    for (int j = 0; j < I; j++) {
      const uint32_t r0 = (uint32_t)(j * P + tid) * V;
      uint32_t f = 0, lanepre = 0, tot = 0;
#pragma unroll
      for (int q = 0; q < V; q++) {
        const bool valid = FULL || ((r0 + q >= rlo) && (r0 + q < rhi));
        const bool left = valid && (ST ? K::lt(key[j][q], pivot) : !K::lt(pivot, key[j][q]));
        if (valid) mn = K::kmin(mn, key[j][q]);
        const uint64_t m = ballot(left);
        lanepre += mbcnt(m);
        tot += __popcll(m);
        f |= (left ? 1u : 0u) << q;
      }
      pre[j] = lanepre;
      flag[j] = f;
      if ((tid & (WAVE - 1)) == 0) sh.cnt[j][w] = tot;
    }
    mn = wave_min<K>(mn);
    if ((tid & (WAVE - 1)) == 0) sh.wmin[w] = mn;
    __syncthreads();
    uint32_t total = 0, mybase[I];
#pragma unroll
    for (int j = 0; j < I; j++) {
      uint32_t before = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ww++) before += (ww < w) ? sh.cnt[j][ww] : 0u;
      mybase[j] = total + before;
#pragma unroll
      for (int ww = 0; ww < NW; ww++) total += sh.cnt[j][ww];
    }
    // the counts are known before the keys are staged: hand them out first
    if (tid == 0) {
      R m2 = sh.wmin[0];
#pragma unroll
      for (int ww = 1; ww < NW; ww++) m2 = K::kmin(m2, sh.wmin[ww]);
      *tmin = m2;
      publish(total, m2);
    }
    const uint32_t nvalid = (uint32_t)(ve - vs);
#pragma unroll
    for (int j = 0; j < I; j++) {
      const uint32_t r0 = (uint32_t)(j * P + tid) * V;
      uint32_t lb = mybase[j] + pre[j];
#pragma unroll
      for (int q = 0; q < V; q++) {
        const uint32_t rv = r0 + q;
        if (FULL || (rv >= rlo && rv < rhi)) {
          const uint32_t pos_in_tile = rv - rlo;
          uint32_t dst;
          if ((flag[j] >> q) & 1u) {
            dst = lb;
            lb++;
          } else {
            const uint32_t rrank = pos_in_tile - lb;   // right keys before this one
            dst = nvalid - 1 - rrank;
          }
          if constexpr (sizeof(S) == sizeof(R)) {
            stage[dst] = key[j][q];
          } else {
            stage[dst] = (S)key[j][q];
          }
        }
      }
    }
    __syncthreads();
    return total;
  }

  // Write the staged tile: stage[0, nleft) to dst[left_base ...] and stage[nleft,
  // nvalid) to dst[right_base ...].  Each run is written in 16-byte aligned chunks of
  // the destination (v-space, off = the arrays' key offset from a 16-byte boundary),
  // one 16-byte store per thread and chunk; only the chunks at the two ends of a run
  // take single-key stores.  tmode != 0 applies the output transform.
  __device__ static void write_out(const S* stage, S* dst, uint32_t nleft, uint32_t nvalid,
                                   uint64_t left_base, uint64_t right_base, int tmode, uint64_t n_total,
                                   int off) {
    write_run(stage, dst, 0, nleft, left_base, tmode, n_total, off);
    write_run(stage, dst, nleft, nvalid - nleft, right_base, tmode, n_total, off);
  }

  // The same with one store per key (each thread writes keys s = tid, tid + P, ...):
  // the workgroup-sequential partitions of the solo kernel measured faster this way.
  __device__ static void write_out_keys(const S* stage, S* dst, uint32_t nleft, uint32_t nvalid,
                                        uint64_t left_base, uint64_t right_base, int tmode, uint64_t n_total) {
    // the two runs in turn; the bounds check is per run (both always hold)
    if (left_base + nleft <= n_total) {
      S* d = dst + left_base;
      for (uint32_t s = threadIdx.x; s < nleft; s += P) d[s] = out_t(stage[s], tmode);
    }
    if (right_base + (nvalid - nleft) <= n_total) {
      S* d = dst + right_base;
      for (uint32_t s = nleft + threadIdx.x; s < nvalid; s += P) d[s - nleft] = out_t(stage[s], tmode);
    }
  }

  __device__ static S out_t(S val, int tmode) {
    if (!tmode) return val;
    R r;
    if constexpr (sizeof(S) == sizeof(R)) {
      r = val;
    } else {
      r = (R)val;
    }
    return K::store_t(r, tmode);
  }

  // (With MIN, also the smallest of the staged keys this thread wrote.)
  template <bool MIN = false>
  __device__ static R write_run(const S* stage, S* dst, uint32_t s0, uint32_t len, uint64_t rb, int tmode,
                                uint64_t n_total, int off) {
    R mn = K::maxv();
    if (len == 0) return mn;
    const uint64_t vb = rb + (uint64_t)off, ve = vb + len;
    const uint64_t c0 = vb / V, c1 = (ve + V - 1) / V;
    char* dbase = reinterpret_cast<char*>(dst - off);   // 16-byte aligned
    for (uint64_t c = c0 + threadIdx.x; c < c1; c += P) {
      const uint64_t v = c * V;
      if (v >= vb && v + V <= ve) {
        const S* from = stage + s0 + (v - vb);
        S tmp[V];
#pragma unroll
        for (int q = 0; q < V; q++) {
          if constexpr (MIN) mn = K::kmin(mn, (R)from[q]);
          tmp[q] = out_t(from[q], tmode);
        }
        uint4 u;
        __builtin_memcpy(&u, tmp, 16);
        *reinterpret_cast<uint4*>(dbase + c * 16) = u;
      } else {
#pragma unroll
        for (int q = 0; q < V; q++) {
          const uint64_t vv = v + q;
          if (vv >= vb && vv < ve) {
            const S x = stage[s0 + (vv - vb)];
            if constexpr (MIN) mn = K::kmin(mn, (R)x);
            if (vv - off < n_total) dst[vv - off] = out_t(x, tmode);
          }
        }
      }
    }
    return mn;
  }

  // write_out that also leaves, per wave, the smallest key written to the right run
  // (K::maxv() for a wave that wrote none) in wrm[w] (LDS), for the next level's
  // planning; visible to the workgroup after its next barrier.
  __device__ static void write_out_rmin(const S* stage, S* dst, uint32_t nleft, uint32_t nvalid,
                                        uint64_t left_base, uint64_t right_base, int tmode, uint64_t n_total,
                                        int off, R* wrm) {
    write_run(stage, dst, 0, nleft, left_base, tmode, n_total, off);
    R m = write_run<true>(stage, dst, nleft, nvalid - nleft, right_base, tmode, n_total, off);
    m = wave_min<K>(m);
    if ((threadIdx.x & (WAVE - 1)) == 0) wrm[threadIdx.x / WAVE] = m;
  }
};

// The tile's smallest right key from the waves' minima (thread 0, after the barrier
// that followed write_out_rmin): stored for the next level's planning.
template <class K>
__device__ inline void store_tile_rmin(const Params& p, unsigned long long g, const typename K::R* wrm) {
  typename K::R m = wrm[0];
#pragma unroll
  for (int w = 1; w < LEVEL_NW; w++) m = K::kmin(m, wrm[w]);
  uint64_t lo, hi;
  K::to_u64x2(m, lo, hi);
  p.tilermin[g].lo = lo;
  p.tilermin[g].hi = hi;
}

// ---- segment bookkeeping --------------------------------------------------------------

__device__ inline void push_solo(const Params& p, const Seg& s) {
  const unsigned long long i = atomicAdd(&p.solo_ctr->count, 1ull);
  if (i >= p.cap_solo) {
    set_err(p, ERR_SOLO_OVERFLOW);
    return;
  }
  p.solo[i] = s;
  atomicAdd(&p.stats->solo_items, 1ull);
}

// A place in a level's range list and its tiles (idx = ~0 on overflow, error set).
template <int T>
__device__ inline void reserve_level(const Params& p, int next_level, const Seg& s, unsigned long long& idx,
                                     unsigned long long& tb) {
  idx = ~0ull;
  tb = 0;
  if (next_level >= p.max_levels - 1) {   // the last level is never launched
    set_err(p, ERR_LEVEL_OVERFLOW);
    return;
  }
  const unsigned long long nt = p.inplace ? ip_tiles_of(s.e - s.b, p.ip_steps) : tiles_of(s.b, s.e, p.off, (uint64_t)T);
  const unsigned long long old = atomicAdd(&p.lvl_ctr[next_level].packed, (1ull << 40) | nt);
  if ((old >> 40) >= p.cap_lvl || (old & TILE_MASK40) + nt > p.cap_tiles) {
    set_err(p, ERR_LEVEL_OVERFLOW);
    return;
  }
  idx = old >> 40;
  tb = old & TILE_MASK40;
}

__device__ inline void write_level(const Params& p, int next_level, const Seg& s, unsigned long long idx,
                                   unsigned long long tb) {
  p.lvl_segs[next_level & 1][idx] = s;
  p.lvl_tbase[next_level & 1][idx] = tb;
  atomicAdd(&p.lvl_ctr[next_level].keys, (unsigned long long)(s.e - s.b));
}

template <class K, int T>
__device__ inline void push_level(const Params& p, int next_level, const Seg& s) {
  unsigned long long idx, tb;
  reserve_level<T>(p, next_level, s, idx, tb);
  if (idx != ~0ull) write_level(p, next_level, s, idx, tb);
}

// Route a range after a partition: short ranges go to the solo list (which checks
// their depth itself), long ones to the next level.  A long range past the paper's
// depth limit continues in fallback mode (counted once as the paper's fallback of
// its length); past the fallback mode's own limit it takes the bounded-time sort.
//
// A range held as runs (run mode) reaches the solo list through a copy entry of the
// next level, which gathers its runs into [b, e) of that level's destination before
// later levels overwrite them.
template <class K, int T>
__device__ inline void to_solo(const Params& p, Seg s, int next_level) {
  if (s.flags & SEG_RUNS) {
    Seg c = s;
    c.flags = (s.flags & (SEG_RUNS | SEG_RIGHT)) | SEG_COPY;
    push_level<K, T>(p, next_level, c);
    const uint32_t keep = SEG_OVERRIDE | SEG_FALLBACK | SEG_BOUNDED | SEG_STRICT;
    s.flags = (s.flags & keep) | ((next_level & 1) ? 0u : SEG_SCRATCH);
  }
  push_solo(p, s);
}

// Where a range goes (the decision only, so that a caller can still give a range
// bound for a level its pivot), then the pushes and counts.
enum : int { RT_NONE = 0, RT_SOLO = 1, RT_LEVEL = 2 };
struct Routed {
  Seg s;
  int dest;
  bool fb_enter;   // enters fallback mode here (counted as the paper's fallback)
};

__device__ inline Routed route_decide(const Params& p, Seg s) {
  Routed r{s, RT_LEVEL, false};
  const uint64_t len = s.e - s.b;
  constexpr uint32_t RUNBITS = SEG_RUNS | SEG_RIGHT;
  if (len == 0) {
    r.dest = RT_NONE;
  } else if (len <= p.solo_max) {
    r.dest = RT_SOLO;
    r.s.flags &= ~(SEG_MAXK | SEG_MINR);
  } else if (s.depth > s.limit) {
    if (!(s.flags & SEG_FALLBACK)) {
      r.fb_enter = true;
      r.s.flags = (s.flags & (SEG_SCRATCH | RUNBITS)) | SEG_FALLBACK;
      r.s.depth = 1;
      r.s.limit = fb_limit_of(p, len);
    }
    if (r.s.depth > r.s.limit) {   // past the fallback mode's own limit
      // (an input range can get here untransformed, with a fallback-mode limit of 0)
      r.s.flags = (s.flags & (SEG_SCRATCH | SEG_RAW | RUNBITS)) | SEG_FALLBACK | SEG_BOUNDED;
      r.dest = RT_SOLO;
    }
  }
  return r;
}

template <class K, int T>
__device__ inline void route_commit(const Params& p, const Routed& r, int next_level) {
  if (r.fb_enter) {
    atomicAdd(&p.stats->fallbacks, 1ull);
    atomicAdd(&p.stats->fallback_keys, (unsigned long long)(r.s.e - r.s.b));
  }
  if (r.dest == RT_SOLO) to_solo<K, T>(p, r.s, next_level);
  else if (r.dest == RT_LEVEL) push_level<K, T>(p, next_level, r.s);
}

template <class K, int T>
__device__ inline void route(const Params& p, Seg s, int next_level) {
  route_commit<K, T>(p, route_decide(p, s), next_level);
}

template <class K>
__device__ inline Seg make_seg(uint64_t b, uint64_t e, uint32_t depth, uint32_t limit, uint32_t flags,
                               typename K::R pv) {
  Seg s{};
  s.b = b;
  s.e = e;
  s.depth = depth;
  s.limit = limit;
  s.flags = flags;
  to_words<K>(pv, s.pv_lo, s.pv_hi);
  return s;
}

static_assert(LEVEL_NW == LEVEL_P / WAVE, "waves of a level workgroup");

// The smallest key of a range routed by the previous level, by a group of G threads
// (gt its index; wsum: G / WAVE words of LDS when G > WAVE): from that level's records
// of the parent's tiles [rt_b, rt_b + rt_n), the tile minima for a left part, the
// tiles' smallest right keys for a right part.
template <class K, int G>
__device__ inline typename K::R range_min(const Params& p, const Seg& sg, int gt, typename K::R* wsum) {
  using R = typename K::R;
  const u128k* tm = ((sg.flags & SEG_MINR) ? p.tilermin : p.tilemin) + sg.rt_b;
  const uint64_t cnt = sg.rt_n;
  constexpr int U = 4;   // loads in flight per thread
  R m[U];
#pragma unroll
  for (int u = 0; u < U; u++) m[u] = K::maxv();
  for (uint64_t t0 = gt; t0 < cnt; t0 += (uint64_t)U * G) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t t = t0 + (uint64_t)u * G;
      if (t < cnt) m[u] = K::kmin(m[u], K::from_u64x2(tm[t].lo, tm[t].hi));
    }
  }
#pragma unroll
  for (int u = 1; u < U; u++) m[0] = K::kmin(m[0], m[u]);
  R r = wave_min<K>(m[0]);
  if constexpr (G > WAVE) {
    if ((gt & (WAVE - 1)) == 0) wsum[gt / WAVE] = r;
    __syncthreads();
    r = wsum[0];
#pragma unroll
    for (int w = 1; w < G / WAVE; w++) r = K::kmin(r, wsum[w]);
    __syncthreads();
  }
  return r;
}

// ---- level kernel ------------------------------------------------------------------------

#ifndef VQS_LB_WIN
#define VQS_LB_WIN 16
#endif
// predecessors a look-back step polls (the wave's first LB_WIN lanes): 16 against 64,
// at four waves per SIMD, 2.5e8 f32 -3.1 %, 2e8 u32 -3.1 %, 2e8 u16 -1.2 % (a step's
// coherent loads cost less, and the nearest inclusive predecessor is usually close)
constexpr int LB_WIN = VQS_LB_WIN;
static_assert(LB_WIN >= 1 && LB_WIN <= WAVE, "look-back window");

// Waves per SIMD the run-mode level kernel is compiled for: as many as its LDS lets in
// (three workgroups of 40 KB tiles per CU for 8-byte keys, four of 32 KB for 16-byte
// keys).  Asking for more than that is not a bound the compiler keeps.
template <int SIZE>
constexpr int runs_waves() { return SIZE == 8 ? 3 : SIZE == 16 ? 4 : 1; }


// Four waves per SIMD (four workgroups per CU) for 2- and 4-byte keys, with 40 and 36
// bytes per lane of spills: 2e8 u16 -7 %, 2.5e8 f32 -3 % and 2e8 u32 -2.4 % (the 4-byte
// kernel spilled 112 bytes at four waves and gained nothing before its ranking lost its
// per-key branch work); the 8- and 16-byte ones fit three and four workgroups by their
// LDS.
template <class K>
__global__ void __launch_bounds__(LEVEL_P) __attribute__((amdgpu_waves_per_eu(K::SIZE <= 4 ? 4 : 1))) level_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int I = K::LI;
  using TL = Tile<K, LEVEL_P, I>;
  constexpr int T = TL::T;
  __shared__ S stage[T];
  __shared__ typename TL::Aux sh;
  __shared__ unsigned long long sh_ticket;
  __shared__ unsigned long long sh_excl;
  __shared__ R sh_segmin;
  __shared__ R sh_wrm[LEVEL_NW];
  __shared__ int sh_seg;
  __shared__ unsigned long long sh_fill0;

  const int L = p.level;
  const unsigned long long packed = p.lvl_ctr[L].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  const unsigned long long ntiles = packed & TILE_MASK40;
  if (ntiles == 0) return;
  const Seg* segs = p.lvl_segs[L & 1];
  const unsigned long long* tbase = p.lvl_tbase[L & 1];
  const bool src_scratch = (L & 1) != 0;
  const S* src = (const S*)(src_scratch ? p.scratch : p.keys);
  S* dst = (S*)(src_scratch ? p.keys : p.scratch);
  const S* src_aligned = src - p.off;
  const int tmode = (L == 0) ? p.mode : 0;   // only the first level reads untransformed keys
  const unsigned long long epoch = (unsigned long long)(L + 1) << 48;
  constexpr unsigned long long ST_AGG = 1ull << 46, ST_INC = 2ull << 46;
  constexpr unsigned long long VAL_MASK = (1ull << 46) - 1;
  const int tid = threadIdx.x;
  unsigned long long tiles_done = 0, keys_done = 0;

  unsigned long long rmin_tile = ~0ull;   // thread 0: tile whose right minimum is pending
  for (;;) {
    if (tid == 0 && rmin_tile != ~0ull) {
      store_tile_rmin<K>(p, rmin_tile, sh_wrm);
      rmin_tile = ~0ull;
    }
    if (tid == 0) sh_ticket = atomicAdd(&p.lvl_ctr[L].ticket, 1u);
    __syncthreads();
    const unsigned long long g = sh_ticket;
    if (g >= ntiles) break;
    // segment of tile g: last s with tbase[s] <= g; one wave narrows the interval
    // 64-fold per step
    if (tid < WAVE) {
      uint32_t lo = 0, hi = nseg;  // invariant: tbase[lo] <= g, and g < tbase[hi] if hi < nseg
      while (hi - lo > 1) {
        const uint32_t span = hi - lo;
        const uint32_t step = (span + WAVE - 1) / WAVE;
        const uint32_t pos = lo + (uint32_t)tid * step;
        const bool le = pos < hi && tbase[pos] <= g;
        const uint64_t m = ballot(le);   // lane 0 always true
        const int last = 63 - __builtin_clzll(m);
        const uint32_t nlo = lo + (uint32_t)last * step;
        const uint32_t nhi = (nlo + step < hi) ? nlo + step : hi;
        lo = nlo;
        hi = nhi;
      }
      if (tid == 0) sh_seg = (int)lo;
    }
    __syncthreads();
    const int si = sh_seg;
    const Seg sg = segs[si];
    if (sg.flags & SEG_SKIP) {   // finished by the planning before this launch
      __syncthreads();
      continue;
    }
    const unsigned long long g0 = tbase[si];
    const uint64_t ntile_seg = tiles_of(sg.b, sg.e, p.off, T);
    const uint64_t k = (sg.b + p.off) / T + (g - g0);
    const uint64_t vs = (k * T > sg.b + p.off) ? k * T : sg.b + p.off;
    const uint64_t ve = ((k + 1) * T < sg.e + p.off) ? (k + 1) * T : sg.e + p.off;
    R key[I][K::V];
    TL::load(src_aligned, k, vs, ve, tmode, key);
    if (sg.flags & SEG_PIVOT) {
      if (tid == 0) sh.pivot = K::from_u64x2(sg.pv_lo, sg.pv_hi);
    } else if (tid < WAVE) {
      const S* sb = src + sg.b;
      R pv = choose_pivot_wave<K>(
          [&](uint64_t i) -> R {
            S s = sb[i];
            R r;
            if constexpr (sizeof(S) == sizeof(R)) r = s; else r = (R)s;
            return tmode ? K::load_t(s, tmode) : r;
          },
          sg.b, sg.e, p);
      if (tid == 0) sh.pivot = pv;
    }
    __syncthreads();
    const R pivot = sh.pivot;
    R tmin;
    // publish the tile minimum, then the left count (the minimum is made visible
    // before the count by waiting for its stores to complete)
    const uint32_t nl = TL::rank_and_stage(stage, sh, key, k, vs, ve, pivot, (sg.flags & SEG_STRICT) != 0, &tmin,
                                           [&](uint32_t cnt, R m) {
                                             uint64_t lo, hi;
                                             to_words<K>(m, lo, hi);
                                             __hip_atomic_store(&p.tilemin[g].lo, lo, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                                             __hip_atomic_store(&p.tilemin[g].hi, hi, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                                             __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                             __builtin_amdgcn_s_waitcnt(0);
                                             __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                             if (g != g0)
                                               __hip_atomic_store(&p.flags[g], epoch | ST_AGG | cnt, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT);
                                           });

    // decoupled look-back on the left counts of the range's earlier tiles, one wave
    // reading 64 predecessors per step
    if (tid < WAVE) {
      const int lane = tid;
      // Only device-coherent single-word accesses are used here (relaxed agent-scope
      // atomics): release/acquire fences at agent scope would write back or
      // invalidate a whole L2 for every tile.
      unsigned long long excl = 0;
      if (g != g0) {
        unsigned long long top = g - 1;   // highest predecessor not yet summed
        uint32_t spins = 0;
        for (;;) {
          const bool inr = lane < LB_WIN && top >= g0 + (unsigned long long)lane;   // lane reads tile top - lane
          unsigned long long f = 0;
          if (inr) f = __hip_atomic_load(&p.flags[top - lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const bool ready = inr && (f & ~((1ull << 48) - 1)) == epoch && (f & (3ull << 46)) != 0;
          const bool inc = ready && (f & ST_INC);
          const uint64_t incm = ballot(inc), readym = ballot(ready), inrm = ballot(inr);
          // lanes up to the nearest inclusive tile must all be ready
          const int first_inc = incm ? __builtin_ctzll(incm) : WAVE;
          const uint64_t need = (first_inc >= WAVE - 1) ? inrm : (((2ull << first_inc) - 1) & inrm);
          if ((need & ~readym) != 0) {
            ++spins;
            if ((spins & 255u) == 0 &&
                (spins > (1u << 20) || __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
              if (lane == 0) set_err(p, ERR_SPIN);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          unsigned long long v = (((need >> lane) & 1ull) != 0) ? (f & VAL_MASK) : 0ull;
#pragma unroll
          for (int m = 1; m < WAVE; m <<= 1) v += (unsigned long long)__shfl_xor((long long)v, m);
          excl += v;
          if (incm) break;
          if (top < g0 + LB_WIN) break;   // cannot happen: tile g0 is always inclusive
          top -= LB_WIN;
        }
      }
      if (lane == 0) {
        __hip_atomic_store(&p.flags[g], epoch | ST_INC | (excl + nl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh_excl = excl;
      }
    }
    __syncthreads();
    const unsigned long long excl_l = sh_excl;
    const uint32_t nvalid = (uint32_t)(ve - vs);
    const uint64_t before = vs - (sg.b + p.off);             // keys of the range before this tile
    const uint64_t excl_r = before - excl_l;
    const uint32_t nr = nvalid - nl;
    TL::write_out_rmin(stage, dst, nl, nvalid, sg.b + excl_l, sg.e - excl_r - nr, 0, p.n_total, p.off, sh_wrm);
    rmin_tile = g;

    if (g == g0 + ntile_seg - 1) {
      // last tile of the range: the range is partitioned; plan what follows
      const uint64_t bound = sg.b + excl_l + nl;
      const bool dst_scratch = !src_scratch;
      const bool fb = (sg.flags & SEG_FALLBACK) != 0;
      const uint32_t cf = (dst_scratch ? SEG_SCRATCH : 0u) | (fb ? SEG_FALLBACK : 0u);
      if (tid == 0) {
        if (!fb) {
          atomicAdd(&p.stats->partitions, 1ull);
          atomicAdd(&p.stats->keys_partitioned, (unsigned long long)(sg.e - sg.b));
          atomicMax(&p.stats->max_depth, (unsigned long long)sg.depth);
        } else {
          atomicAdd(&p.stats->fallback_partitions, 1ull);
        }
      }
      // keys of [fb_, fe_) all equal the pivot and are final.  The caller's array holds
      // them already unless it holds transformed keys there (whole range: it holds the
      // range's keys in some order), or, for a part of the range, unless the partition
      // wrote the caller's array (otherwise it holds the unpartitioned range)
      auto retire_equal = [&](uint64_t fb_, uint64_t fe_, bool part) {
        const bool need = part ? (dst_scratch || p.mode != 0) : (p.mode != 0 && L > 0);
        if (!need || fe_ <= fb_) return;
        const uint64_t nch = (fe_ - fb_ + FILL_CHUNK - 1) / FILL_CHUNK;
        if (tid == 0) {
          sh_fill0 = atomicAdd(&p.solo_ctr->count, (unsigned long long)nch);
          atomicAdd(&p.stats->solo_items, (unsigned long long)nch);
        }
        __syncthreads();
        uint64_t lo, hi;
        to_words<K>(pivot, lo, hi);
        for (uint64_t c = tid; c < nch; c += LEVEL_P) {
          const unsigned long long i = sh_fill0 + c;
          if (i >= p.cap_solo) {
            set_err(p, ERR_SOLO_OVERFLOW);
            continue;
          }
          Seg f{};
          f.b = fb_ + c * FILL_CHUNK;
          f.e = (f.b + FILL_CHUNK < fe_) ? f.b + FILL_CHUNK : fe_;
          f.flags = SEG_FILL;
          f.pv_lo = lo;
          f.pv_hi = hi;
          p.solo[i] = f;
        }
      };
      if (sg.flags & SEG_STRICT) {
        // fallback mode after a degenerate partition: [b, bound) holds the keys before
        // the pivot, [bound, e) the keys equal to it, which are final
        retire_equal(bound, sg.e, true);
        if (tid == 0) route<K, T>(p, make_seg<K>(sg.b, bound, sg.depth + 1, sg.limit, cf, pivot), L + 1);
      } else if (bound == sg.e && !fb) {
        // degenerate: the minimum of the range decides (Alg. 1, ScanMinMax)
        R m = K::maxv();
        for (unsigned long long t = g0 + tid; t <= g; t += LEVEL_P) {
          const uint64_t wlo = __hip_atomic_load(&p.tilemin[t].lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t whi = __hip_atomic_load(&p.tilemin[t].hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          m = K::kmin(m, K::from_u64x2(wlo, whi));
        }
        m = wave_min<K>(m);
        if ((tid & (WAVE - 1)) == 0) sh.wmin[tid / WAVE] = m;
        __syncthreads();
        if (tid == 0) {
          R mm = sh.wmin[0];
          for (int ww = 1; ww < LEVEL_P / WAVE; ww++) mm = K::kmin(mm, sh.wmin[ww]);
          sh_segmin = mm;
        }
        __syncthreads();
        const R mn = sh_segmin;
        if (tid == 0) atomicAdd(&p.stats->degenerate, 1ull);
        if (K::eq(mn, pivot)) {
          if (tid == 0) atomicAdd(&p.stats->all_equal, 1ull);
          retire_equal(sg.b, sg.e, false);
        } else if (tid == 0) {
          // the range's largest key is the pivot (every key went left)
          Seg r = make_seg<K>(sg.b, sg.e, sg.depth + 1, sg.limit, cf | SEG_OVERRIDE | SEG_PIVOT | SEG_MAXK, mn);
          to_words<K>(pivot, r.mx_lo, r.mx_hi);
          route<K, T>(p, r, L + 1);
        }
      } else if (bound == sg.e) {
        // fallback mode, degenerate: split off the keys equal to the pivot (the maximum)
        if (tid == 0)
          route<K, T>(p, make_seg<K>(sg.b, sg.e, sg.depth + 1, sg.limit, cf | SEG_OVERRIDE | SEG_PIVOT | SEG_STRICT, pivot),
                      L + 1);
      } else if (tid == 0) {
        Seg lc = make_seg<K>(sg.b, bound, sg.depth + 1, sg.limit, cf, pivot);
        Seg rc = make_seg<K>(bound, sg.e, sg.depth + 1, sg.limit, cf, pivot);
        if (!fb) {
          // for the next level's planning: the left part's largest key is the pivot (a key
          // of the range, and keys equal to it go left), the right part's is the range's
          // when that is known; their minima come from this level's records of the
          // range's tiles [g0, g0 + ntile_seg) (range_min)
          lc.flags |= SEG_MAXK;
          to_words<K>(pivot, lc.mx_lo, lc.mx_hi);
          rc.flags |= SEG_MINR | (sg.flags & SEG_MAXK);
          rc.mx_lo = sg.mx_lo;
          rc.mx_hi = sg.mx_hi;
          lc.rt_b = rc.rt_b = (uint32_t)g0;
          lc.rt_n = rc.rt_n = (uint32_t)ntile_seg;
        }
        route<K, T>(p, lc, L + 1);
        route<K, T>(p, rc, L + 1);
      }
    }
    tiles_done++;
    keys_done += nvalid;
    __syncthreads();
  }
  if (tid == 0 && tiles_done) {
    atomicAdd(&p.stats->level_tiles, tiles_done);
    atomicAdd(&p.stats->hbm_read_keys, keys_done);
    atomicAdd(&p.stats->hbm_write_keys, keys_done);
  }
}

// ---- run mode: ranges held as runs of the previous level's tiles --------------------
//
// In run mode a level tile writes its partition into its own interval of the
// destination (left keys in input order, then the right keys in reverse input order),
// so no tile waits for another.  A child range is then the concatenation of one run
// per tile of its parent: the left child takes the tiles' left parts in tile order,
// the right child their right parts in reverse tile order.  That is the key sequence
// the contiguous partition writes, so pivots and the recursion are unchanged.  The
// planning launch after the partition records every tile's run starts inside both
// children (TileRun) and, for each tile of the next level, its range and first run.

// start (child-relative) of run u of a run-held range, and the source position of its
// first key
__device__ inline void run_info(const TileRun* tab, const Seg& s, uint64_t u, uint64_t& start, uint64_t& first) {
  const bool right = (s.flags & SEG_RIGHT) != 0;
  const TileRun& r = tab[right ? (uint64_t)s.rt_b + (s.rt_n - 1 - u) : (uint64_t)s.rt_b + u];
  start = right ? r.rp : r.lp;
  first = right ? r.pos + r.nl : r.pos;
}

__device__ inline uint64_t run_start(const TileRun* tab, const Seg& s, uint64_t u) {
  const bool right = (s.flags & SEG_RIGHT) != 0;
  return right ? tab[(uint64_t)s.rt_b + (s.rt_n - 1 - u)].rp : tab[(uint64_t)s.rt_b + u].lp;
}

// source position of key j (child-relative) of a run-held range: the last run starting
// at or before j (runs may be empty; the last one starting at or before a valid j is not)
__device__ inline uint64_t run_pos(const TileRun* tab, const Seg& s, uint64_t j, uint64_t lo = 0) {
  uint64_t hi = s.rt_n;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) / 2;
    if (run_start(tab, s, mid) <= j) lo = mid;
    else hi = mid;
  }
  uint64_t st, first;
  run_info(tab, s, lo, st, first);
  return first + (j - st);
}

__device__ inline uint64_t wave_incl_scan64(uint64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), d);
    if (lane >= d) v += ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// one entry per run a tile touches: key at tile slot s of run i sits at mbase + s
struct RunEnt {
  int64_t mbase;
  int32_t rst;   // first tile slot of the run (0 for the run holding slot 0)
  int32_t pad;
};

// Level partition in run mode: the same tiles, classification, ranks and LDS staging
// as level_kernel, but each tile writes its interval [vs, ve) of the destination, so
// there is no look-back.  A tile of a run-held range reads its keys through the runs
// (the runs it touches are listed in LDS first).  Each tile leaves its left count and
// minimum; runs_plan_kernel plans the ranges afterwards.  Copy entries only gather
// their runs into [b, e) for the solo kernel.
template <class K>
__global__ void __launch_bounds__(LEVEL_P) __attribute__((amdgpu_waves_per_eu(runs_waves<sizeof(typename K::R)>()))) level_runs_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int I = K::LI;
  using TL = Tile<K, LEVEL_P, I>;
  constexpr int T = TL::T;
  constexpr int TC = TL::TC;
  constexpr int V = K::V;
  constexpr int NW = LEVEL_P / WAVE;
  constexpr int RMAX = (int)(T * sizeof(S) / sizeof(RunEnt));
  __shared__ __align__(16) S stage[T];
  __shared__ typename TL::Aux sh;
  __shared__ unsigned long long sh_tk[2];
  __shared__ R sh_wrm[LEVEL_NW];
  __shared__ int sh_seg;
  RunEnt* ent = reinterpret_cast<RunEnt*>(stage);

  const int L = p.level;
  const unsigned long long packed = p.lvl_ctr[L].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  const unsigned long long ntiles = packed & TILE_MASK40;
  if (ntiles == 0) return;
  Seg* segs = p.lvl_segs[L & 1];
  const unsigned long long* tbase = p.lvl_tbase[L & 1];
  const bool src_scratch = (L & 1) != 0;
  const S* src = (const S*)(src_scratch ? p.scratch : p.keys);
  S* dst = (S*)(src_scratch ? p.keys : p.scratch);
  const S* src_aligned = src - p.off;
  const int tmode = (L == 0) ? p.mode : 0;   // only the first level reads untransformed keys
  const TileRun* prev = p.runs[(L + 1) & 1];
  const int tid = threadIdx.x;
  unsigned long long tiles_done = 0, keys_done = 0;

  // tiles are independent: the next tile's ticket is drawn when a tile starts, and
  // handed over through alternating LDS slots at its end
  if (tid == 0) sh_tk[0] = atomicAdd(&p.lvl_ctr[L].ticket, 1u);
  __syncthreads();
  unsigned long long rmin_tile = ~0ull;   // thread 0: tile whose right minimum is pending
  for (int it = 0;; it++) {
    if (tid == 0 && rmin_tile != ~0ull) {
      store_tile_rmin<K>(p, rmin_tile, sh_wrm);
      rmin_tile = ~0ull;
    }
    const unsigned long long g = sh_tk[it & 1];
    if (g >= ntiles) break;
    unsigned int g_next = 0;
    if (tid == 0) g_next = atomicAdd(&p.lvl_ctr[L].ticket, 1u);
    // a planned level records each tile's range (and first run); the input ranges of
    // the first level are found by search
    const bool planned = L != p.seed_level;
    TileRef tr{0, 0};
    if (planned) tr = p.tref[g];
    if (!planned && tid < WAVE) {
      uint32_t lo = 0, hi = nseg;  // invariant: tbase[lo] <= g, and g < tbase[hi] if hi < nseg
      while (hi - lo > 1) {
        const uint32_t span = hi - lo;
        const uint32_t step = (span + WAVE - 1) / WAVE;
        const uint32_t pos = lo + (uint32_t)tid * step;
        const bool le = pos < hi && tbase[pos] <= g;
        const uint64_t m = ballot(le);   // lane 0 always true
        const int last = 63 - __builtin_clzll(m);
        const uint32_t nlo = lo + (uint32_t)last * step;
        const uint32_t nhi = (nlo + step < hi) ? nlo + step : hi;
        lo = nlo;
        hi = nhi;
      }
      if (tid == 0) sh_seg = (int)lo;
    }
    if (!planned) __syncthreads();
    const int si = planned ? (int)tr.seg : sh_seg;
    const Seg sg = segs[si];
    if (sg.flags & SEG_SKIP) {   // finished by the planning launch: no keys to move
      if (tid == 0) sh_tk[(it + 1) & 1] = g_next;
      __syncthreads();
      continue;
    }
    const unsigned long long g0 = tbase[si];
    const uint64_t nt = tiles_of(sg.b, sg.e, p.off, T);
    const uint64_t k = (sg.b + p.off) / T + (g - g0);
    const uint64_t vs = (k * T > sg.b + p.off) ? k * T : sg.b + p.off;
    const uint64_t ve = ((k + 1) * T < sg.e + p.off) ? (k + 1) * T : sg.e + p.off;
    const uint32_t nvalid = (uint32_t)(ve - vs);

    R key[I][V];
    if (!(sg.flags & SEG_RUNS)) {
      TL::load(src_aligned, k, vs, ve, tmode, key);
    } else {
      // the runs the tile touches into LDS (from the first one, recorded by the
      // planning launch), then every key from its run
      const uint64_t j0 = vs - p.off - sg.b, j1 = j0 + nvalid;
      const uint64_t u0 = tr.frun;   // recorded by the planning launch
      uint32_t nr = 0;
      for (uint32_t r = 0;; r++) {
        const uint64_t u = u0 + (uint64_t)r * LEVEL_P + tid;
        bool in = false;
        if (u < sg.rt_n) {
          uint64_t st, first;
          run_info(prev, sg, u, st, first);
          in = st < j1 || u == u0;
          const uint32_t idx = r * LEVEL_P + tid;
          if (in && idx < (uint32_t)RMAX) {
            ent[idx].rst = st <= j0 ? 0 : (int32_t)(st - j0);
            ent[idx].mbase = (int64_t)first - (int64_t)st + (int64_t)j0;
          }
        }
        const int cnt = __syncthreads_count(in);
        nr += (uint32_t)cnt;
        if (cnt < LEVEL_P) break;
      }
      S raw[I][V];
      if (nr <= (uint32_t)RMAX) {
        // a thread's slots increase with (j, q): walk the run list forward
        int i = 0;
        int32_t nxt = nr > 1 ? ent[1].rst : INT32_MAX;
        int64_t mb = ent[0].mbase;
#pragma unroll
        for (int j = 0; j < I; j++) {
#pragma unroll
          for (int q = 0; q < V; q++) {
            const uint64_t v = (k * TC + (uint64_t)j * LEVEL_P + tid) * V + q;
            const int32_t sl = v < vs ? 0 : (v >= ve ? (int32_t)nvalid - 1 : (int32_t)(v - vs));
            while (sl >= nxt) {
              i++;
              mb = ent[i].mbase;
              nxt = (i + 1 < (int)nr) ? ent[i + 1].rst : INT32_MAX;
            }
            raw[j][q] = src[mb + sl];
          }
        }
      } else {
        // more runs than the LDS list holds: search each key's run, in sequence into
        // LDS, then read the tile from there
        for (uint32_t sl = tid; sl < nvalid; sl += LEVEL_P) stage[sl] = src[run_pos(prev, sg, j0 + sl, u0)];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < I; j++) {
#pragma unroll
          for (int q = 0; q < V; q++) {
            const uint64_t v = (k * TC + (uint64_t)j * LEVEL_P + tid) * V + q;
            raw[j][q] = stage[v < vs ? 0 : (v >= ve ? nvalid - 1 : v - vs)];
          }
        }
      }
      if (sg.flags & SEG_COPY) {
        // gather only: the keys in sequence to [vs, ve) of the destination
        char* dbase = reinterpret_cast<char*>(dst - p.off);
#pragma unroll
        for (int j = 0; j < I; j++) {
          const uint64_t c = k * TC + (uint64_t)j * LEVEL_P + tid;
          const uint64_t v0 = c * V;
          if (v0 >= vs && v0 + V <= ve) {
            uint4 u;
            __builtin_memcpy(&u, raw[j], 16);
            *reinterpret_cast<uint4*>(dbase + c * 16) = u;
          } else {
#pragma unroll
            for (int q = 0; q < V; q++)
              if (v0 + q >= vs && v0 + q < ve) dst[v0 + q - p.off] = raw[j][q];
          }
        }
        tiles_done++;
        keys_done += nvalid;
        if (tid == 0) sh_tk[(it + 1) & 1] = g_next;
        __syncthreads();   // the LDS run list is read before the next tile rewrites it
        continue;
      }
#pragma unroll
      for (int j = 0; j < I; j++) {
#pragma unroll
        for (int q = 0; q < V; q++) {
          if constexpr (sizeof(S) == sizeof(R)) {
            key[j][q] = raw[j][q];
          } else {
            key[j][q] = (R)raw[j][q];
          }
        }
      }
    }
    // the planning launch gave every range of the level its pivot
    if (tid == 0) {
      sh.pivot = K::from_u64x2(sg.pv_lo, sg.pv_hi);
      if (!(sg.flags & SEG_PIVOT)) set_err(p, ERR_NO_PIVOT);
    }
    __syncthreads();   // also: the LDS run list is read before the keys are staged over it
    const R pivot = sh.pivot;
    R tmin;
    // the tile's left count and minimum, for the planning launch after this one
    const uint32_t nl = TL::rank_and_stage(stage, sh, key, k, vs, ve, pivot, (sg.flags & SEG_STRICT) != 0, &tmin,
                                           [&](uint32_t cnt, R m) {
                                             uint64_t lo, hi;
                                             to_words<K>(m, lo, hi);
                                             p.tilemin[g].lo = lo;
                                             p.tilemin[g].hi = hi;
                                             p.tnl[g] = cnt;
                                           });
    TL::write_out_rmin(stage, dst, nl, nvalid, vs - p.off, vs - p.off + nl, 0, p.n_total, p.off, sh_wrm);
    rmin_tile = g;
    tiles_done++;
    keys_done += nvalid;
    if (tid == 0) sh_tk[(it + 1) & 1] = g_next;
    __syncthreads();
  }
  if (tid == 0 && tiles_done) {
    atomicAdd(&p.stats->level_tiles, tiles_done);
    atomicAdd(&p.stats->hbm_read_keys, keys_done);
    atomicAdd(&p.stats->hbm_write_keys, keys_done);
  }
}

// ---- run mode: planning ------------------------------------------------------------

template <class K>
struct PlanShared {
  static constexpr int W = 64 / K::SIZE;   // keys per ChoosePivot chunk
  unsigned long long wsum[LEVEL_P / WAVE];
  uint64_t o[2][9];                       // the children's ChoosePivot chunk starts
  uint64_t spos[2][9 * W];                // source positions of their sampled keys
  typename K::R wmin[LEVEL_P / WAVE];
  typename K::R pv[2];
  typename K::R mn[2];                    // minima of children with a foreseen degenerate partition
  typename K::R samp[2][9 * W];           // the sampled keys
};

// recursion counts of a planning group, added to the device totals once per workgroup
struct PlanCounts {
  unsigned long long part, pkeys, maxd, deg, alleq, fbpart, fbs, fbkeys, solo, lvlkeys;
};

// What the first half of a range's planning leaves for the second: the thread's left
// keys before its tiles and in them, the range's left count, the routed children, the fills, and
// what the range needs of the level and solo lists (reserved in between, for several
// ranges at once).
struct PlanState {
  uint64_t lp0, myl, ltot;
  Routed r0, r1;
  uint64_t fill_b, fill_e, nfill, nsolo, nt0, nt1;
  uint32_t ne;   // level entries (0, 1 or 2)
  bool degenerate, all_equal, piv0, piv1;
};

// where the reservations put a range's entries
struct PlanSlots {
  unsigned long long idx, tb, solo;   // idx = ~0: no level entries (or an overflow)
};

// a range record made wave-uniform (scalar registers)
__device__ inline Seg uniform_seg(const Seg& s) {
  Seg u;
  const uint32_t* a = reinterpret_cast<const uint32_t*>(&s);
  uint32_t* b = reinterpret_cast<uint32_t*>(&u);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(Seg) / 4); i++) b[i] = __builtin_amdgcn_readfirstlane(a[i]);
  return u;
}

// barrier of a planning group: the workgroup, or one wave
template <int G>
__device__ inline void gsync() {
  if constexpr (G == WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int G>
__device__ inline uint64_t group_excl_scan(uint64_t v, uint64_t& total, unsigned long long* wsum, int gt) {
  const uint64_t incl = wave_incl_scan64(v);
  if constexpr (G == WAVE) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)incl, WAVE - 1);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(incl >> 32), WAVE - 1);
    total = uniform64(((uint64_t)hi << 32) | lo);
    return incl - v;
  } else {
    const int w = gt / WAVE;
    if ((gt & (WAVE - 1)) == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t ex = incl - v;
    total = 0;
#pragma unroll
    for (int ww = 0; ww < G / WAVE; ww++) {
      ex += (ww < w) ? wsum[ww] : 0ull;
      total += wsum[ww];
    }
    total = uniform64(total);
    __syncthreads();
    return ex;
  }
}

// one reservation of the level list and one of the solo list for a batch of ranges
// (thread 0); returns the first slots
__device__ inline PlanSlots plan_reserve(const Params& p, int L, unsigned long long ne, unsigned long long ntiles,
                                         unsigned long long nsolo) {
  PlanSlots r{~0ull, 0, 0};
  if (ne) {
    if (L >= p.max_levels - 1) {   // the last level is never launched
      set_err(p, ERR_LEVEL_OVERFLOW);
    } else {
      const unsigned long long old = atomicAdd(&p.lvl_ctr[L].packed, (ne << 40) | ntiles);
      if ((old >> 40) + ne > p.cap_lvl || (old & TILE_MASK40) + ntiles > p.cap_tiles) {
        set_err(p, ERR_LEVEL_OVERFLOW);
      } else {
        r.idx = old >> 40;
        r.tb = old & TILE_MASK40;
      }
    }
  }
  if (nsolo) r.solo = atomicAdd(&p.solo_ctr->count, nsolo);
  return r;
}

// Planning of one range of level L-1 after its partition, by a group of G threads
// (the workgroup, or one wave for a range of few tiles); gt is the thread's index in
// the group.  First half: the tiles' left counts give the bound; the children are
// routed as in level_kernel.
template <class K, int G>
__device__ PlanState plan_first(const Params& p, int L, const Seg& sg, uint64_t g0, uint64_t nt, PlanShared<K>& sm,
                                int gt) {
  using R = typename K::R;
  constexpr int I = K::LI;
  constexpr int T = Tile<K, LEVEL_P, I>::T;
  const TileRun* tab = p.runs[(L - 1) & 1];
  const bool dst_scratch = ((L - 1) & 1) == 0;   // where level L-1 wrote
  const R pivot = K::from_u64x2(sg.pv_lo, sg.pv_hi);
  PlanState st{};
  // the range's left count (each thread a block of consecutive tiles)
  const uint64_t per = (nt + G - 1) / G;
  const uint64_t ta = (uint64_t)gt * per < nt ? (uint64_t)gt * per : nt;
  const uint64_t tb = ta + per < nt ? ta + per : nt;
  constexpr int QB = G == WAVE ? 4 : 16;   // counts read per batch, all in flight
  const uint32_t* tnl = p.tnl;
  uint64_t sl = 0;
  for (uint64_t a = ta; a < tb; a += QB) {
    uint32_t cv[QB];
#pragma unroll
    for (int q = 0; q < QB; q++) cv[q] = tnl[g0 + ((a + q < tb) ? a + q : a)];
#pragma unroll
    for (int q = 0; q < QB; q++) sl += (a + q < tb) ? cv[q] : 0u;
  }
  st.lp0 = group_excl_scan<G>(sl, st.ltot, sm.wsum, gt);
  st.myl = sl;
  const uint64_t bound = sg.b + st.ltot;
  const bool fb = (sg.flags & SEG_FALLBACK) != 0;
  const uint32_t cf = (dst_scratch ? SEG_SCRATCH : 0u) | (fb ? SEG_FALLBACK : 0u);
  // the children (child 0 holds the tiles' left parts, child 1 their right parts)
  auto child = [&](uint64_t b, uint64_t e, uint32_t flags, R pv, bool right) {
    Seg c = make_seg<K>(b, e, sg.depth + 1, sg.limit, flags | SEG_RUNS | (right ? SEG_RIGHT : 0u), pv);
    c.rt_b = (uint32_t)g0;
    c.rt_n = (uint32_t)nt;
    return c;
  };
  int nc = 0;
  Seg c0{}, c1{};
  if (sg.flags & SEG_STRICT) {
    // fallback mode after a degenerate partition: [b, bound) holds the keys before
    // the pivot, [bound, e) the keys equal to it
    st.fill_b = bound;
    st.fill_e = sg.e;
    c0 = child(sg.b, bound, cf, pivot, false);
    nc = 1;
  } else if (bound == sg.e && !fb) {
    // degenerate: the minimum of the range decides (Alg. 1, ScanMinMax)
    st.degenerate = true;
    Seg whole{};   // the range's own tiles of level L-1
    whole.rt_b = (uint32_t)g0;
    whole.rt_n = (uint32_t)nt;
    const R mn = range_min<K, G>(p, whole, gt, sm.wmin);
    if (K::eq(mn, pivot)) {
      st.all_equal = true;
      st.fill_b = sg.b;
      st.fill_e = sg.e;
    } else {
      // the range's largest key is the pivot (every key went left)
      c0 = child(sg.b, sg.e, cf | SEG_OVERRIDE | SEG_PIVOT | SEG_MAXK, mn, false);
      to_words<K>(pivot, c0.mx_lo, c0.mx_hi);
      nc = 1;
    }
  } else if (bound == sg.e) {
    // fallback mode, degenerate: split off the keys equal to the pivot (the maximum)
    c0 = child(sg.b, sg.e, cf | SEG_OVERRIDE | SEG_PIVOT | SEG_STRICT, pivot, false);
    nc = 1;
  } else {
    c0 = child(sg.b, bound, cf, pivot, false);
    c1 = child(bound, sg.e, cf, pivot, true);
    if (!fb) {
      // largest keys, for foreseeing degenerate partitions (as in level_kernel)
      c0.flags |= SEG_MAXK;
      to_words<K>(pivot, c0.mx_lo, c0.mx_hi);
      c1.flags |= SEG_MINR | (sg.flags & SEG_MAXK);
      c1.mx_lo = sg.mx_lo;
      c1.mx_hi = sg.mx_hi;
    }
    nc = 2;
  }
  st.r0 = route_decide(p, c0);
  st.r1 = route_decide(p, c1);
  if (nc < 1) st.r0.dest = RT_NONE;
  if (nc < 2) st.r1.dest = RT_NONE;
  // every child is held as runs: each gets tiles at level L (itself, or its copy entry)
  st.ne = (st.r0.dest != RT_NONE ? 1u : 0u) + (st.r1.dest != RT_NONE ? 1u : 0u);
  st.nt0 = st.r0.dest != RT_NONE ? tiles_of(st.r0.s.b, st.r0.s.e, p.off, T) : 0;
  st.nt1 = st.r1.dest != RT_NONE ? tiles_of(st.r1.s.b, st.r1.s.e, p.off, T) : 0;
  st.piv0 = st.r0.dest == RT_LEVEL && !(st.r0.s.flags & SEG_PIVOT);
  st.piv1 = st.r1.dest == RT_LEVEL && !(st.r1.s.flags & SEG_PIVOT);
  st.nfill = st.fill_e > st.fill_b ? (st.fill_e - st.fill_b + FILL_CHUNK - 1) / FILL_CHUNK : 0;
  st.nsolo = (st.r0.dest == RT_SOLO ? 1 : 0) + (st.r1.dest == RT_SOLO ? 1 : 0) + st.nfill;
  return st;
}

// Second half: every tile's run starts in the children (TileRun); the first run of
// each child tile at level L; ChoosePivot of each child bound for level L without a
// given pivot (its nine chunk starts are drawn, the pass over the tiles records where
// the sampled keys sit, then they are read together); the level and solo entries at
// the reserved slots; counts go to pc (thread 0 of the group).
template <class K, int G>
__device__ void plan_second(const Params& p, int L, const Seg& sg, uint64_t g0, uint64_t nt, PlanShared<K>& sm,
                            int gt, const PlanState& st, const PlanSlots& sl_, PlanCounts& pc) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int I = K::LI;
  constexpr int T = Tile<K, LEVEL_P, I>::T;
  constexpr int W = PlanShared<K>::W;
  TileRun* tab = p.runs[(L - 1) & 1];
  const S* src_next = (const S*)((L & 1) ? p.scratch : p.keys);   // what level L reads
  const R pivot = K::from_u64x2(sg.pv_lo, sg.pv_hi);
  const uint64_t off = (uint64_t)p.off;
  const bool fb = (sg.flags & SEG_FALLBACK) != 0;
  const Routed& r0 = st.r0;
  const Routed& r1 = st.r1;
  const bool ok = sl_.idx != ~0ull;
  const bool have0 = r0.dest != RT_NONE && ok, have1 = r1.dest != RT_NONE && ok;
  const uint64_t tb_0 = sl_.tb, tb_1 = sl_.tb + st.nt0;
  if (gt < 2 && (gt == 0 ? st.piv0 : st.piv1)) {
    const Seg& cc = gt == 0 ? r0.s : r1.s;
    uint64_t o[9];
    pivot_chunk_starts<K>(cc.b, cc.e, p, o);
#pragma unroll
    for (int i = 0; i < 9; i++) sm.o[gt][i] = o[i];
  }
  gsync<G>();
  const uint64_t per = (nt + G - 1) / G;
  const uint64_t ta = (uint64_t)gt * per < nt ? (uint64_t)gt * per : nt;
  const uint64_t tb = ta + per < nt ? ta + per : nt;
  const uint64_t rtot = (sg.e - sg.b) - st.ltot;
  // the sampled chunks that meet this thread's part of each child: its left parts are
  // [lp0, lp0 + its left keys) of child 0, its right parts [rlo, rhi) of child 1
  uint32_t cm0 = 0, cm1 = 0;
  if (st.piv0 || st.piv1) {
    const uint64_t kb = (sg.b + off) / T;
    const uint64_t kbs = (kb + ta) * T > sg.b + off ? (kb + ta) * T : sg.b + off;
    const uint64_t kbe = (kb + tb) * T < sg.e + off ? (kb + tb) * T : sg.e + off;
    const uint64_t mine = tb > ta ? kbe - kbs : 0;                        // keys of my tiles
    const uint64_t before = tb > ta ? kbs - (sg.b + off) : 0;             // keys of earlier tiles
    const uint64_t myl = st.myl;
    const uint64_t rhi = rtot - (before - st.lp0), rlo = rhi - (mine - myl);
#pragma unroll
    for (int ch = 0; ch < 9; ch++) {
      if (st.piv0 && sm.o[0][ch] < st.lp0 + myl && sm.o[0][ch] + W > st.lp0) cm0 |= 1u << ch;
      if (st.piv1 && sm.o[1][ch] < rhi && sm.o[1][ch] + W > rlo) cm1 |= 1u << ch;
    }
  }
  // first runs of the child tiles: a thread's left parts are contiguous in child 0 and
  // its right parts in child 1 (in reverse tile order), so it walks the child tile
  // starts forward through child 0 and backward through child 1.  Child tile m starts
  // at 0 (m = 0) or at (kc + m) * T - off - b.
  auto tile_start = [&](const Seg& cc, uint64_t m) -> uint64_t {
    return m == 0 ? 0 : ((cc.b + off) / T + m) * T - off - cc.b;
  };
  const uint32_t cseg0 = (uint32_t)sl_.idx, cseg1 = (uint32_t)(sl_.idx + (r0.dest != RT_NONE ? 1 : 0));
  uint64_t m0 = 0, s0 = 0;   // next child-0 tile and its start
  int64_t m1 = -1;           // next child-1 tile (downward)
  uint64_t s1 = 0;
  if (have0 && st.lp0 > 0) {
    m0 = (st.lp0 + r0.s.b + off + T - 1) / T - (r0.s.b + off) / T;
    s0 = m0 < st.nt0 ? tile_start(r0.s, m0) : 0;
  }
  if (have1) {
    const uint64_t kb = (sg.b + off) / T;
    const uint64_t kbs = (kb + ta) * T > sg.b + off ? (kb + ta) * T : sg.b + off;
    const uint64_t before = tb > ta ? kbs - (sg.b + off) : 0;
    const uint64_t rhi = rtot - (before - st.lp0);   // end of my right parts in child 1
    if (rhi > 0) {
      int64_t m = (int64_t)((rhi + r1.s.b + off + T - 1) / T - (r1.s.b + off) / T) - 1;
      if (m > (int64_t)st.nt1 - 1) m = (int64_t)st.nt1 - 1;
      m1 = m;
      s1 = m1 >= 0 ? tile_start(r1.s, (uint64_t)m1) : 0;
    }
  }
  constexpr int QB = G == WAVE ? 4 : 16;
  const uint32_t* tnl = p.tnl;
  uint64_t lp = st.lp0;
  for (uint64_t a = ta; a < tb; a += QB) {
    uint32_t cv[QB];
#pragma unroll
    for (int q = 0; q < QB; q++) cv[q] = tnl[g0 + ((a + q < tb) ? a + q : a)];
#pragma unroll
    for (int q = 0; q < QB; q++) {
      if (a + q >= tb) break;
      const uint64_t t = a + q;
      const uint64_t kk = (sg.b + off) / T + t;
      const uint64_t tvs = (kk * T > sg.b + off) ? kk * T : sg.b + off;
      const uint64_t tve = ((kk + 1) * T < sg.e + off) ? (kk + 1) * T : sg.e + off;
      const uint64_t nv = tve - tvs;
      const uint64_t before = tvs - (sg.b + off);   // keys of the range's earlier tiles
      TileRun tr;
      tr.lp = lp;
      tr.rp = rtot - ((before + nv) - (lp + cv[q]));   // right keys of later tiles
      tr.pos = tvs - off;
      tr.nl = cv[q];
      tr.nv = (uint32_t)nv;
      tab[g0 + t] = tr;
      lp += cv[q];
#pragma unroll 1
      for (int side = 0; side < 2; side++) {
        const bool have = side == 0 ? have0 : have1;
        const uint32_t cm = side == 0 ? cm0 : cm1;
        if (!have && !cm) continue;
        const Seg& cc = side == 0 ? r0.s : r1.s;
        // this tile's run in the child: [rs, rs + rl), first key at src_next[first]
        const uint64_t rs = side == 0 ? tr.lp : tr.rp;
        const uint64_t rl = side == 0 ? tr.nl : nv - tr.nl;
        const uint64_t first = side == 0 ? tr.pos : tr.pos + tr.nl;
        if (rl == 0) continue;
        if (side == 0 && have) {
          // child-0 tiles starting in [rs, rs + rl)
          while (m0 < st.nt0 && s0 < rs + rl) {
            p.tref[tb_0 + m0] = TileRef{cseg0, (uint32_t)t};
            m0++;
            s0 = m0 == 1 ? tile_start(cc, 1) : s0 + T;
          }
        } else if (side == 1 && have) {
          // child-1 tiles starting in [rs, rs + rl) (runs come downward)
          while (m1 >= 0 && s1 >= rs) {
            p.tref[tb_1 + (uint64_t)m1] = TileRef{cseg1, (uint32_t)(nt - 1 - t)};
            m1--;
            s1 = m1 <= 0 ? 0 : s1 - T;
          }
        }
        for (uint32_t mm = cm; mm; mm &= mm - 1) {
          const int ch = __builtin_ctz(mm);
          const uint64_t o = sm.o[side][ch];
          const uint64_t lo = o > rs ? o : rs;
          const uint64_t hi = (o + W < rs + rl) ? o + W : rs + rl;
          for (uint64_t i = lo; i < hi; i++) sm.spos[side][ch * W + (i - o)] = first + (i - rs);
        }
      }
    }
  }
  gsync<G>();
  // the sampled keys, all loads in flight together, then ChoosePivot of each child
  if (st.piv0 || st.piv1) {
    for (int k = gt; k < 2 * 9 * W; k += G) {
      const int side = k / (9 * W), j = k % (9 * W);
      if (side == 0 ? st.piv0 : st.piv1) {
        const S sv = src_next[sm.spos[side][j]];
        R rv;
        if constexpr (sizeof(S) == sizeof(R)) rv = sv; else rv = (R)sv;
        sm.samp[side][j] = rv;
      }
    }
    gsync<G>();
    auto lds_pivot = [&](int side) {
      return choose_pivot_from<K>([&](uint64_t i) -> R { return sm.samp[side][i]; }, 0, W, 2 * W, 3 * W, 4 * W,
                                  5 * W, 6 * W, 7 * W, 8 * W);
    };
    if constexpr (G == WAVE) {
      if (st.piv0) {
        const R v = lds_pivot(0);
        if (gt == 0) sm.pv[0] = v;
      }
      if (st.piv1) {
        const R v = lds_pivot(1);
        if (gt == 0) sm.pv[1] = v;
      }
    } else {
      const int w = gt / WAVE;
      if (w < 2 && (w == 0 ? st.piv0 : st.piv1)) {
        const R v = lds_pivot(w);
        if ((gt & (WAVE - 1)) == 0) sm.pv[w] = v;
      }
    }
    gsync<G>();
  }
  // degenerate partitions foreseen (see pivot_kernel): a child whose pivot is its known
  // largest key; its minimum, by the group
  bool fd[2] = {false, false};
  {
#pragma unroll
    for (int side = 0; side < 2; side++) {
      const Routed& r = side == 0 ? r0 : r1;
      fd[side] = (side == 0 ? st.piv0 : st.piv1) && ok && (r.s.flags & SEG_MAXK) && !(r.s.flags & SEG_FALLBACK) &&
                 K::eq(sm.pv[side], K::from_u64x2(r.s.mx_lo, r.s.mx_hi));
    }
    if (fd[0] || fd[1]) {
#pragma unroll
      for (int side = 0; side < 2; side++) {
        if (fd[side]) {
          const R m = range_min<K, G>(p, side == 0 ? r0.s : r1.s, gt, sm.wmin);
          if (gt == 0) sm.mn[side] = m;
        }
      }
      gsync<G>();
    }
  }
  if (gt == 0) {
    if (!fb) {
      pc.part++;
      pc.pkeys += sg.e - sg.b;
      pc.maxd = sg.depth > pc.maxd ? sg.depth : pc.maxd;
    } else {
      pc.fbpart++;
    }
    pc.deg += st.degenerate ? 1 : 0;
    pc.alleq += st.all_equal ? 1 : 0;
    pc.solo += st.nsolo;
    unsigned long long si = sl_.solo, li = sl_.idx;
#pragma unroll
    for (int side = 0; side < 2; side++) {
      Routed r = side == 0 ? r0 : r1;
      if (r.dest == RT_NONE) continue;
      if (r.fb_enter) {
        pc.fbs++;
        pc.fbkeys += r.s.e - r.s.b;
      }
      if ((side == 0 ? st.piv0 : st.piv1)) {
        to_words<K>(sm.pv[side], r.s.pv_lo, r.s.pv_hi);
        r.s.flags |= SEG_PIVOT;
      }
      bool skip = false;
      if (fd[side]) {
        // the foreseen degenerate partition, counted as the oracle counts it; then the
        // range is all one value (filled, its level entry skipped) or is partitioned
        // again with its minimum as pivot, one level deeper (unless past the limit)
        const R pv = sm.pv[side], mn = sm.mn[side];
        if (K::eq(mn, pv) || r.s.depth + 1 <= r.s.limit) {
          pc.part++;
          pc.pkeys += r.s.e - r.s.b;
          pc.maxd = r.s.depth > pc.maxd ? r.s.depth : pc.maxd;
          pc.deg++;
        }
        if (K::eq(mn, pv)) {
          pc.alleq++;
          skip = true;
          const uint64_t nch = (r.s.e - r.s.b + FILL_CHUNK - 1) / FILL_CHUNK;
          const unsigned long long f0 = atomicAdd(&p.solo_ctr->count, (unsigned long long)nch);
          pc.solo += nch;
          for (uint64_t c = 0; c < nch; c++) {
            if (f0 + c >= p.cap_solo) {
              set_err(p, ERR_SOLO_OVERFLOW);
              break;
            }
            Seg f{};
            f.b = r.s.b + c * FILL_CHUNK;
            f.e = (f.b + FILL_CHUNK < r.s.e) ? f.b + FILL_CHUNK : r.s.e;
            f.flags = SEG_FILL;
            to_words<K>(pv, f.pv_lo, f.pv_hi);
            p.solo[f0 + c] = f;
          }
        } else if (r.s.depth + 1 <= r.s.limit) {
          to_words<K>(mn, r.s.pv_lo, r.s.pv_hi);
          r.s.depth += 1;
          r.s.flags |= SEG_OVERRIDE;
        }
      }
      if (ok) {
        // the range itself, or the copy entry that gathers it for the solo list
        Seg e = r.s;
        if (r.dest == RT_SOLO) e.flags = (r.s.flags & (SEG_RUNS | SEG_RIGHT)) | SEG_COPY;
        if (skip) e.flags |= SEG_SKIP;
        p.lvl_segs[L & 1][li] = e;
        p.lvl_tbase[L & 1][li] = side == 0 ? tb_0 : tb_1;
        if (!skip) pc.lvlkeys += e.e - e.b;
        li++;
      }
      if (r.dest == RT_SOLO) {
        // gathered into [b, e) of level L's destination by the copy entry
        Seg so = r.s;
        const uint32_t keep = SEG_OVERRIDE | SEG_FALLBACK | SEG_BOUNDED | SEG_STRICT;
        so.flags = (r.s.flags & keep) | ((L & 1) ? 0u : SEG_SCRATCH);
        if (si < p.cap_solo) p.solo[si] = so;
        else set_err(p, ERR_SOLO_OVERFLOW);
        si++;
      }
    }
  }
  // keys equal to the pivot are final: fill entries of the solo list write them (they
  // follow the range's other solo entries)
  if (st.nfill) {
    const unsigned long long f0 = sl_.solo + st.nsolo - st.nfill;
    uint64_t lo, hi;
    to_words<K>(pivot, lo, hi);
    for (uint64_t c = gt; c < st.nfill; c += G) {
      const unsigned long long i = f0 + c;
      if (i >= p.cap_solo) {
        set_err(p, ERR_SOLO_OVERFLOW);
        continue;
      }
      Seg f{};
      f.b = st.fill_b + c * FILL_CHUNK;
      f.e = (f.b + FILL_CHUNK < st.fill_e) ? f.b + FILL_CHUNK : st.fill_e;
      f.flags = SEG_FILL;
      f.pv_lo = lo;
      f.pv_hi = hi;
      p.solo[i] = f;
    }
  }
  gsync<G>();
}

// Run mode, before the partition launch of level L: plan every range of level L-1:
// ranges of many tiles by a workgroup each, the others by a wave each, four at a time
// per workgroup so that one reservation of each list serves four ranges.  At the first
// level, the input ranges get their pivots (one wave per range).
template <class K>
__global__ void __launch_bounds__(LEVEL_P) runs_plan_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int I = K::LI;
  constexpr int T = Tile<K, LEVEL_P, I>::T;
  constexpr int NW = LEVEL_P / WAVE;
  constexpr uint64_t SMALL = 4 * WAVE;   // ranges of at most this many tiles: one wave each
  __shared__ PlanShared<K> smg;
  __shared__ PlanShared<K> smw[NW];
  __shared__ unsigned long long need[NW][3];
  __shared__ PlanSlots slots[NW];
  __shared__ unsigned long long cnt_sh[10];
  const int L = p.level;
  const int tid = threadIdx.x;
  const int w = tid / WAVE;
  const int lane = tid & (WAVE - 1);
  if (L == p.seed_level) {
    const unsigned long long packed = p.lvl_ctr[L].packed;
    const uint32_t nseg = (uint32_t)(packed >> 40);
    Seg* segs = p.lvl_segs[L & 1];
    const S* src = (const S*)((L & 1) ? p.scratch : p.keys);
    const int tmode = (L == 0) ? p.mode : 0;
    const uint32_t nwaves = gridDim.x * NW;
    for (uint32_t si = blockIdx.x * NW + w; si < nseg; si += nwaves) {
      const Seg sg = segs[si];
      if (sg.flags & (SEG_OVERRIDE | SEG_PIVOT)) continue;
      const S* sb = src + sg.b;
      const R pv = choose_pivot_wave<K>(
          [&](uint64_t i) -> R {
            S sv = sb[i];
            R r;
            if constexpr (sizeof(S) == sizeof(R)) r = sv; else r = (R)sv;
            return tmode ? K::load_t(sv, tmode) : r;
          },
          sg.b, sg.e, p);
      if (lane == 0) {
        uint64_t lo, hi;
        to_words<K>(pv, lo, hi);
        segs[si].pv_lo = lo;
        segs[si].pv_hi = hi;
        segs[si].flags = sg.flags | SEG_PIVOT;
      }
    }
    return;
  }
  const int LP = L - 1;
  const unsigned long long packed = p.lvl_ctr[LP].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  if ((packed & TILE_MASK40) == 0) return;
  const Seg* segs = p.lvl_segs[LP & 1];
  const unsigned long long* tbase = p.lvl_tbase[LP & 1];
  if (tid < 10) cnt_sh[tid] = 0;
  PlanCounts pc{};
  for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
    const Seg sg = uniform_seg(segs[si]);
    const uint64_t nt = tiles_of(sg.b, sg.e, p.off, T);
    if ((sg.flags & (SEG_COPY | SEG_SKIP)) || nt <= SMALL) continue;   // gathers and finished ranges: no plan
    const uint64_t g0 = uniform64(tbase[si]);
    const PlanState st = plan_first<K, LEVEL_P>(p, L, sg, g0, nt, smg, tid);
    if (tid == 0) slots[0] = plan_reserve(p, L, st.ne, st.nt0 + st.nt1, st.nsolo);
    __syncthreads();
    const PlanSlots sl_ = slots[0];
    plan_second<K, LEVEL_P>(p, L, sg, g0, nt, smg, tid, st, sl_, pc);
  }
  for (uint32_t base = blockIdx.x * NW; base < nseg; base += gridDim.x * NW) {
    const uint32_t si = base + w;
    Seg sg{};
    uint64_t nt = 0, g0 = 0;
    bool mine = false;
    if (si < nseg) {
      sg = uniform_seg(segs[si]);
      nt = tiles_of(sg.b, sg.e, p.off, T);
      mine = !(sg.flags & (SEG_COPY | SEG_SKIP)) && nt <= SMALL;
      g0 = uniform64(tbase[si]);
    }
    PlanState st{};
    if (mine) st = plan_first<K, WAVE>(p, L, sg, g0, nt, smw[w], lane);
    if (lane == 0) {
      need[w][0] = mine ? st.ne : 0;
      need[w][1] = mine ? st.nt0 + st.nt1 : 0;
      need[w][2] = mine ? st.nsolo : 0;
    }
    __syncthreads();
    if (tid == 0) {
      const PlanSlots s0 = plan_reserve(p, L, need[0][0] + need[1][0] + need[2][0] + need[3][0],
                                        need[0][1] + need[1][1] + need[2][1] + need[3][1],
                                        need[0][2] + need[1][2] + need[2][2] + need[3][2]);
      unsigned long long di = 0, dt = 0, ds = 0;
      for (int ww = 0; ww < NW; ww++) {
        slots[ww].idx = (s0.idx == ~0ull || need[ww][0] == 0) ? ~0ull : s0.idx + di;
        slots[ww].tb = s0.tb + dt;
        slots[ww].solo = s0.solo + ds;
        di += need[ww][0];
        dt += need[ww][1];
        ds += need[ww][2];
      }
    }
    __syncthreads();
    if (mine) plan_second<K, WAVE>(p, L, sg, g0, nt, smw[w], lane, st, slots[w], pc);
    __syncthreads();
  }
  // the workgroup's counts: one device atomic each
  __syncthreads();
  if (lane == 0) {
    const unsigned long long v[9] = {pc.part, pc.pkeys, pc.deg, pc.alleq, pc.fbpart,
                                     pc.fbs, pc.fbkeys, pc.solo, pc.lvlkeys};
#pragma unroll
    for (int i = 0; i < 9; i++)
      if (v[i]) atomicAdd(&cnt_sh[i], v[i]);
    if (pc.maxd) atomicMax(&cnt_sh[9], pc.maxd);
  }
  __syncthreads();
  if (tid == 0) {
    if (cnt_sh[0]) atomicAdd(&p.stats->partitions, cnt_sh[0]);
    if (cnt_sh[1]) atomicAdd(&p.stats->keys_partitioned, cnt_sh[1]);
    if (cnt_sh[2]) atomicAdd(&p.stats->degenerate, cnt_sh[2]);
    if (cnt_sh[3]) atomicAdd(&p.stats->all_equal, cnt_sh[3]);
    if (cnt_sh[4]) atomicAdd(&p.stats->fallback_partitions, cnt_sh[4]);
    if (cnt_sh[5]) atomicAdd(&p.stats->fallbacks, cnt_sh[5]);
    if (cnt_sh[6]) atomicAdd(&p.stats->fallback_keys, cnt_sh[6]);
    if (cnt_sh[7]) atomicAdd(&p.stats->solo_items, cnt_sh[7]);
    if (cnt_sh[8]) atomicAdd(&p.lvl_ctr[L].keys, cnt_sh[8]);
    if (cnt_sh[9]) atomicMax(&p.stats->max_depth, cnt_sh[9]);
  }
}

// ChoosePivot for every range of a level, one wave per range, before the level's
// partition launch: the tiles then read the pivot with the range record.
//
// Degenerate partitions are foreseen here.  With pivot pv, a range's partition is
// degenerate exactly when pv is its largest key, which the range record carries when
// it is known (a left part's largest key is its parent's pivot, a right part inherits
// its parent's).  Alg. 1 then finds the range's minimum and stops if it equals pv (all
// keys equal), else partitions again with the minimum as pivot, one level deeper.
// Since a partition that sends every key left leaves the keys where and as they were,
// neither step needs this level's pass: the minimum is reduced from what the previous
// level recorded for the range's parent (range_min), the partition is counted as the
// oracle counts it, and the range either leaves the level (filled with its one value)
// or becomes that second partition.  A second partition past the depth limit takes the
// level pass.
constexpr int PIVOT_P = 256;

template <class K>
__global__ void __launch_bounds__(PIVOT_P) pivot_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  const int L = p.level;
  const unsigned long long packed = p.lvl_ctr[L].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  if (nseg == 0) return;
  Seg* segs = p.lvl_segs[L & 1];
  const S* src = (const S*)((L & 1) && !p.inplace ? p.scratch : p.keys);
  const int tmode = (L == 0) ? p.mode : 0;
  const uint32_t wave = (blockIdx.x * PIVOT_P + threadIdx.x) / WAVE;
  const uint32_t nwaves = gridDim.x * (PIVOT_P / WAVE);
  for (uint32_t si = wave; si < nseg; si += nwaves) {
    const Seg sg = segs[si];
    if (sg.flags & (SEG_OVERRIDE | SEG_PIVOT)) continue;
    const S* sb = src + sg.b;
    const R pv = choose_pivot_wave<K>(
        [&](uint64_t i) -> R {
          S sv = sb[i];
          R r;
          if constexpr (sizeof(S) == sizeof(R)) r = sv; else r = (R)sv;
          return tmode ? K::load_t(sv, tmode) : r;
        },
        sg.b, sg.e, p);
    {
      if (L > 0 && (sg.flags & SEG_MAXK) && !(sg.flags & SEG_FALLBACK) &&
          K::eq(pv, K::from_u64x2(sg.mx_lo, sg.mx_hi))) {
        const R mn = range_min<K, WAVE>(p, sg, lane_id(), nullptr);
        const uint64_t len = sg.e - sg.b;
        if (K::eq(mn, pv)) {
          // all keys equal: the caller's array holds them already unless the level reads
          // scratch or the keys are transformed
          if (lane_id() == 0) {
            atomicAdd(&p.stats->partitions, 1ull);
            atomicAdd(&p.stats->keys_partitioned, (unsigned long long)len);
            atomicMax(&p.stats->max_depth, (unsigned long long)sg.depth);
            atomicAdd(&p.stats->degenerate, 1ull);
            atomicAdd(&p.stats->all_equal, 1ull);
            atomicAdd(&p.lvl_ctr[L].keys, 0ull - (unsigned long long)len);   // keys the pass moves
            segs[si].flags = sg.flags | SEG_SKIP;
          }
          if ((L & 1) != 0 || p.mode != 0) {
            const uint64_t nch = (len + FILL_CHUNK - 1) / FILL_CHUNK;
            unsigned long long f0 = 0;
            if (lane_id() == 0) {
              f0 = atomicAdd(&p.solo_ctr->count, (unsigned long long)nch);
              atomicAdd(&p.stats->solo_items, (unsigned long long)nch);
            }
            f0 = __shfl(f0, 0);
            for (uint64_t c = lane_id(); c < nch; c += WAVE) {
              const unsigned long long i = f0 + c;
              if (i >= p.cap_solo) {
                set_err(p, ERR_SOLO_OVERFLOW);
                continue;
              }
              Seg f{};
              f.b = sg.b + c * FILL_CHUNK;
              f.e = (f.b + FILL_CHUNK < sg.e) ? f.b + FILL_CHUNK : sg.e;
              f.flags = SEG_FILL;
              to_words<K>(pv, f.pv_lo, f.pv_hi);
              p.solo[i] = f;
            }
          }
          continue;
        }
        if (sg.depth + 1 <= sg.limit) {
          if (lane_id() == 0) {
            atomicAdd(&p.stats->partitions, 1ull);
            atomicAdd(&p.stats->keys_partitioned, (unsigned long long)len);
            atomicMax(&p.stats->max_depth, (unsigned long long)sg.depth);
            atomicAdd(&p.stats->degenerate, 1ull);
            uint64_t lo, hi;
            to_words<K>(mn, lo, hi);
            segs[si].pv_lo = lo;
            segs[si].pv_hi = hi;
            segs[si].depth = sg.depth + 1;
            segs[si].flags = sg.flags | SEG_OVERRIDE | SEG_PIVOT;
          }
          continue;
        }
      }
    }
    if (lane_id() == 0) {
      uint64_t lo, hi;
      to_words<K>(pv, lo, hi);
      segs[si].pv_lo = lo;
      segs[si].pv_hi = hi;
      segs[si].flags = sg.flags | SEG_PIVOT;
    }
  }
}

// ---- base case: 16x16 sorting network in registers (Sec. 2.3, Sec. 3) ------------------

// Green's 16-input network: four hypercube layers, then 28 modules.
#define VQS_GREEN16(CE)                                                                            \
  CE(0, 1) CE(2, 3) CE(4, 5) CE(6, 7) CE(8, 9) CE(10, 11) CE(12, 13) CE(14, 15)                  \
  CE(0, 2) CE(1, 3) CE(4, 6) CE(5, 7) CE(8, 10) CE(9, 11) CE(12, 14) CE(13, 15)                  \
  CE(0, 4) CE(1, 5) CE(2, 6) CE(3, 7) CE(8, 12) CE(9, 13) CE(10, 14) CE(11, 15)                  \
  CE(0, 8) CE(1, 9) CE(2, 10) CE(3, 11) CE(4, 12) CE(5, 13) CE(6, 14) CE(7, 15)                  \
  CE(5, 10) CE(6, 9) CE(3, 12) CE(13, 14) CE(7, 11) CE(1, 2) CE(4, 8)                            \
  CE(1, 4) CE(7, 13) CE(2, 8) CE(11, 14) CE(5, 6) CE(9, 10)                                      \
  CE(2, 4) CE(11, 13) CE(3, 8) CE(7, 12)                                                          \
  CE(6, 8) CE(10, 12) CE(3, 5) CE(7, 9)                                                           \
  CE(3, 4) CE(5, 6) CE(7, 8) CE(9, 10) CE(11, 12)                                                 \
  CE(6, 7) CE(8, 9)

// Sorts 16 registers x 16 lanes of each 16-lane group: the group's 256 keys end in
// sequence order s = 16 * (lane % 16) + register.  Column sort: Green's network in
// every lane (no lane traffic).  Merges of adjacent groups of w lanes: the flip stage
// pairs lane l, register r with lane l ^ (2w-1), register 15-r, bringing the two nodes
// of every module to the same register of two lanes; half-cleaners at lane distances
// w/2..1 exchange the same register; the last four stages are inside each lane.
template <class K, int W>
__device__ inline void merge_stage16(typename K::R (&x)[16], int gl) {
  using R = typename K::R;
  // A lane keeps the smaller key of its pair (up = false) or the larger (up = true):
  // it takes the partner's key y when (y before x) differs from up; for equal keys it
  // may take y, which is the same key.  One compare per key.
  // flip stage: lane l, register r  <->  lane l ^ (2W-1), register 15-r
  {
    const bool up = (gl & W) != 0;
    // registers r and 15-r in pairs: two temporaries instead of sixteen
#pragma unroll
    for (int r = 0; r < 8; r++) {
      const R ya = xor_lanes<2 * W - 1>(x[15 - r]);
      const R yb = xor_lanes<2 * W - 1>(x[r]);
      x[r] = K::sel(K::lt(ya, x[r]) != up, ya, x[r]);
      x[15 - r] = K::sel(K::lt(yb, x[15 - r]) != up, yb, x[15 - r]);
    }
  }
  // half-cleaners across lanes (distance W/2 .. 1)
  auto cross = [&](auto dtag) {
    constexpr int D = decltype(dtag)::value;
    const bool up = (gl & D) != 0;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      R y = xor_lanes<D>(x[r]);
      x[r] = K::sel(K::lt(y, x[r]) != up, y, x[r]);
    }
  };
  if constexpr (W >= 8) cross(std::integral_constant<int, 4>{});
  if constexpr (W >= 4) cross(std::integral_constant<int, 2>{});
  if constexpr (W >= 2) cross(std::integral_constant<int, 1>{});
  // half-cleaners inside each lane (register distance 8, 4, 2, 1)
#pragma unroll
  for (int d = 8; d >= 1; d /= 2) {
#pragma unroll
    for (int r = 0; r < 16; r++)
      if ((r & d) == 0) {
        const bool sw = K::lt(x[r + d], x[r]);
        const R lo = K::sel(sw, x[r + d], x[r]);
        const R hi = K::sel(sw, x[r], x[r + d]);
        x[r] = lo;
        x[r + d] = hi;
      }
  }
}

template <class K>
__device__ inline void network16x16(typename K::R (&x)[16]) {
  using R = typename K::R;
  const int gl = lane_id() & 15;
#define VQS_CE(a, b)                     \
  {                                      \
    const bool sw_ = K::lt(x[b], x[a]);  \
    const R lo_ = K::sel(sw_, x[b], x[a]); \
    const R hi_ = K::sel(sw_, x[a], x[b]); \
    x[a] = lo_;                          \
    x[b] = hi_;                          \
  }
  VQS_GREEN16(VQS_CE)
#undef VQS_CE
  merge_stage16<K, 1>(x, gl);
  merge_stage16<K, 2>(x, gl);
  merge_stage16<K, 4>(x, gl);
  merge_stage16<K, 8>(x, gl);
}

// ---- local sort in LDS (workgroup) --------------------------------------------------------

constexpr int SOLO_NW = SOLO_P / WAVE;
constexpr int LIST_CAP = LOCAL_LIST_CAP;
constexpr int BC_CAP = 256;     // base cases per LDS recursion level

// LDS item flags
enum : uint32_t {
  LI_INB = 1u,       // the range's keys are in buffer B
  LI_OVERRIDE = 2u,  // pivot given
  LI_FB = 4u,        // fallback mode (past the paper's depth limit)
  LI_STRICT = 8u,    // split into keys before the pivot and keys equal to it
};

template <class K>
struct LocalItem {
  uint32_t lb, le;
  uint32_t depth, limit;
  uint32_t flags;
  typename K::R pv;
};

// The recursion counts of a solo workgroup (its local sorts and its partitions through
// device memory), summed in LDS by its thread 0 and added to the device-wide counters
// once, when the solo kernel ends.
struct LocalCounts {
  unsigned long long part, pkeys, bc, deg, eq, fb, fbkeys, maxd;
  unsigned long long gpart, gkeys, fbpart;   // the solo kernel's partitions through device memory
};

template <class K>
struct LocalShared {
  LocalItem<K> list[2][LIST_CAP];
  uint32_t bc[BC_CAP];          // lb << 10 | (len-1) << 2 | fallback-mode << 1 | in B
  LocalItem<K> bounded[LIST_CAP];  // ranges past the fallback-mode limit
  uint32_t pvoff[2][LIST_CAP][9];          // the ranges' ChoosePivot chunk starts
  typename K::R gpiv[SOLO_NW / 2], gmin[SOLO_NW];   // wave groups: pivots, part minima
  uint32_t gcnt[SOLO_NW];                  // wave groups: left counts of the parts
  uint32_t nlist[2];
  uint32_t nbc, nbounded;
  uint32_t stat_part, stat_bc, stat_deg, stat_eq, stat_fb, stat_fbkeys, stat_maxd, stat_pkeys;
};

// Bitonic sort (flip form: every module puts the smaller key at the lower index) of
// a[0, n) in LDS by the whole workgroup; virtual positions >= n act as +inf and never
// move, so no padding is stored.  Bounded time; used for ranges that exceed the
// fallback mode's own depth limit.
template <class K, class S>
__device__ void wg_bitonic_lds(S* a, uint32_t n) {
  using R = typename K::R;
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (uint32_t kk = 2; kk <= p2; kk <<= 1) {
    for (uint32_t d = kk; d >= 2; d >>= 1) {
      const uint32_t half = d >> 1;
      for (uint32_t idx = threadIdx.x; idx < p2 / 2; idx += blockDim.x) {
        const uint32_t i = (idx / half) * d + (idx % half);
        const uint32_t j = (d == kk) ? (i ^ (d - 1)) : (i + half);
        if (j < n) {
          R x = (R)a[i], y = (R)a[j];
          if (K::lt(y, x)) {
            a[i] = (S)y;
            a[j] = (S)x;
          }
        }
      }
      __syncthreads();
    }
  }
}

#include "vqs_inplace.h"

// Sort keys [b, e) of `src` (n <= local_cap) in LDS and write them to `out` (the
// caller's array, output transform applied) or, if out_internal, to `out` in internal
// form.  bufA/bufB hold local_cap keys each.  item_flags: LI_OVERRIDE / LI_FB /
// LI_STRICT of the range (pv is the given pivot).
//
// Past the paper's depth limit (where its Heapsort runs) a range continues in fallback
// mode: same partitions, but a degenerate partition is repeated with the strict
// predicate "key before pivot", which splits off every key equal to the pivot (the
// range's maximum) at once; a fallback-mode range deeper than its own limit
// 2*log2(len)+4 is sorted by the bounded-time bitonic network.  Work in fallback mode
// is not counted as the paper's partitions or base cases (the paper's fallback is one
// leaf); entering it is counted as one fallback of the range's length.
template <class K, bool IP>
__device__ void local_sort(const Params& p, LocalShared<K>& ls, typename K::S* bufA, typename K::S* bufB,
                           const typename K::S* src, bool raw, uint64_t b, uint64_t e, uint32_t depth,
                           uint32_t limit, uint32_t item_flags, typename K::R pv, typename K::S* out,
                           bool out_internal, LocalCounts& acc) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int V = K::V;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / WAVE;
  const uint32_t n = (uint32_t)(e - b);
  const int tmode = raw ? p.mode : 0;

  // 1. load into bufA[0, n) (16-byte aligned chunks in v-space).  A thread's chunks
  // are all requested before any is used (a chunk past the range reads the range's
  // last one, a safe address, and is dropped), and the first pivot's chunk starts are
  // drawn meanwhile.
  const S* src_aligned = src - p.off;
  const uint64_t vb = b + p.off, ve = e + p.off;
  const uint64_t c0 = vb / V, c1 = (ve + V - 1) / V;
  constexpr int LC = (LOCAL_BYTES / 16 + 1 + SOLO_P - 1) / SOLO_P;   // chunks per thread at most
  uint4 rawc[LC];
  if (c1 > c0) {
#pragma unroll
    for (int j = 0; j < LC; j++) {
      uint64_t c = c0 + tid + (uint64_t)j * SOLO_P;
      c = c < c1 ? c : c1 - 1;
      rawc[j] = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(src_aligned) + c * 16);
    }
  }
  if (tid == 0) {
    ls.nlist[0] = 0;
    ls.nlist[1] = 0;
    ls.nbc = 0;
    ls.nbounded = 0;
    ls.stat_part = ls.stat_bc = ls.stat_deg = ls.stat_eq = ls.stat_fb = ls.stat_fbkeys = ls.stat_maxd = 0;
    ls.stat_pkeys = 0;
    if (n > 0) {
      if (n <= p.nb) {
        ls.bc[0] = (0u << 10) | ((n - 1) << 2) | ((item_flags & LI_FB) ? 2u : 0u);
        ls.nbc = 1;
      } else {
        LocalItem<K> it;
        it.lb = 0;
        it.le = n;
        it.depth = depth;
        it.limit = limit;
        it.flags = item_flags & (LI_OVERRIDE | LI_FB | LI_STRICT);
        it.pv = pv;
        ls.list[0][0] = it;
        ls.nlist[0] = 1;
        uint64_t o[9];
        pivot_chunk_starts<K>(b, e, p, o);
#pragma unroll
        for (int i = 0; i < 9; i++) ls.pvoff[0][0][i] = (uint32_t)o[i];
      }
    }
  }
  if (c1 > c0) {
    // range position of chunk c's first key: (c - c0) * V - head (32-bit)
    const uint32_t head = (uint32_t)(vb - c0 * V), nch = (uint32_t)(c1 - c0);
#pragma unroll
    for (int j = 0; j < LC; j++) {
      const uint32_t ci = (uint32_t)tid + (uint32_t)j * SOLO_P;
      if (ci < nch) {
        R tmp[V];
        K::unpack(rawc[j], tmp);
        const int32_t r0 = (int32_t)(ci * V) - (int32_t)head;
#pragma unroll
        for (int q = 0; q < V; q++) {
          const int32_t ri = r0 + q;
          if (ri >= 0 && (uint32_t)ri < n) {
            R r = tmp[q];
            if (tmode) r = K::load_t((S)r, tmode);
            bufA[ri] = (S)r;
          }
        }
      }
    }
  }
  __syncthreads();

  // this wave's recursion counts (wave-uniform), added to the workgroup's at the end
  uint32_t w_part = 0, w_pkeys = 0, w_maxd = 0, w_deg = 0, w_eq = 0;
  int cur = 0;
  for (;;) {
    const uint32_t nitems = ls.nlist[cur];
    // 2. partition this level's ranges: one wave per range, or, while there are at
    // most half as many ranges as waves, G waves per range (the largest power of two
    // with nitems * G <= waves)
    int G = 1;
    while (nitems > 0 && 2u * G * nitems <= (uint32_t)SOLO_NW) G *= 2;
    // depth check of an item: true if it is to be partitioned (possibly now in
    // fallback mode); false if it went to the bounded-time list (by lane 0 of the
    // wave that reports it)
    auto admit = [&](LocalItem<K>& it, bool report) -> bool {
      if (it.depth <= it.limit) return true;
      const uint32_t lb = it.lb, le = it.le;
      if (!(it.flags & LI_FB)) {
        // the paper's depth limit: continue this range in fallback mode
        if (report && lane == 0) {
          atomicAdd(&ls.stat_fb, 1u);
          atomicAdd(&ls.stat_fbkeys, le - lb);
        }
        it.flags = (it.flags & LI_INB) | LI_FB;
        it.depth = 1;
        it.limit = fb_limit_of(p, le - lb);
        if (it.depth <= it.limit) return true;
      }
      if (report && lane == 0) {
        const uint32_t f = atomicAdd(&ls.nbounded, 1u);
        if (f < LIST_CAP) ls.bounded[f] = it;
        else set_err(p, ERR_LOCAL_OVERFLOW);
      }
      return false;
    };
    // ChoosePivot from the chunk starts computed for the level's ranges in advance
    auto pick_pivot = [&](const LocalItem<K>& it, uint32_t idx, const S* s_buf) -> R {
      if (it.flags & LI_OVERRIDE) return it.pv;
      const S* sb = s_buf + it.lb;
      const uint32_t* o = ls.pvoff[cur][idx];
      return choose_pivot_from<K>([&](uint64_t i) -> R { return (R)sb[i]; }, o[0], o[1], o[2], o[3], o[4], o[5],
                                  o[6], o[7], o[8]);
    };
    // after the partition of it into d_buf ([lb, bound) left): children, equal runs,
    // statistics.  Run by one whole wave; mn is the range minimum (wave-uniform).
    auto plan = [&](const LocalItem<K>& it, uint32_t bound, R mn, R pivot) {
      const uint32_t lb = it.lb, le = it.le;
      const bool fb = (it.flags & LI_FB) != 0;
      const bool strict = (it.flags & LI_STRICT) != 0;
      const uint32_t nbuf = (it.flags & LI_INB) ? 0u : LI_INB;   // children live in d_buf
      if (!fb) {
        w_part++;
        w_pkeys += le - lb;
        w_maxd = it.depth > w_maxd ? it.depth : w_maxd;
      }
      auto push_child = [&](uint32_t cb, uint32_t ce, uint32_t cflags, R cpv) {
        const uint32_t len = ce - cb;
        if (len == 0) return;
        if (len <= p.nb) {
          const uint32_t s = atomicAdd(&ls.nbc, 1u);
          if (s < BC_CAP) ls.bc[s] = (cb << 10) | ((len - 1) << 2) | (fb ? 2u : 0u) | (nbuf ? 1u : 0u);
          else set_err(p, ERR_LOCAL_OVERFLOW);
        } else {
          LocalItem<K> ci;
          ci.lb = cb;
          ci.le = ce;
          ci.depth = it.depth + 1;
          ci.limit = it.limit;
          ci.flags = nbuf | (fb ? LI_FB : 0u) | cflags;
          ci.pv = cpv;
          const uint32_t s = atomicAdd(&ls.nlist[cur ^ 1], 1u);
          if (s < LIST_CAP) ls.list[cur ^ 1][s] = ci;
          else set_err(p, ERR_LOCAL_OVERFLOW);
        }
      };
      auto finish_equal = [&](uint32_t cb, uint32_t ce) {
        // all keys of [cb, ce) are equal: done; they must sit in bufA
        if (nbuf)
          for (uint32_t i = cb + lane; i < ce; i += WAVE) bufA[i] = bufB[i];
      };
      if (strict) {
        // [lb, bound): keys before the pivot; [bound, le): keys equal to it
        finish_equal(bound, le);
        if (lane == 0) push_child(lb, bound, 0u, pivot);
      } else if (bound == le) {
        if (!fb) {
          w_deg++;
          if (K::eq(mn, pivot)) {
            w_eq++;
            finish_equal(lb, le);
          } else if (lane == 0) {
            // Alg. 1: repeat with the first key in sort order as the pivot
            push_child(lb, le, LI_OVERRIDE, mn);
          }
        } else if (lane == 0) {
          // fallback mode: split off the keys equal to the pivot (the maximum)
          push_child(lb, le, LI_OVERRIDE | LI_STRICT, pivot);
        }
      } else if (lane < 2) {
        // both children at once (their LDS atomics issue as one instruction)
        push_child(lane == 0 ? lb : bound, lane == 0 ? bound : le, 0u, pivot);
      }
    };
    constexpr int U = 4;   // four 64-key groups per step: independent loads, ballots, stores
    // Keys of [pb, pe) to d_buf: left keys in order from l, right keys in order downward
    // from r - 1; returns the final l.  The predicate (left: not after the pivot, or
    // before it for a strict split) is fixed per instantiation, and whole steps of U
    // vectors need no bounds: only the tail's last vector is partial.
    auto scatter = [&](auto strict_tag, const S* s_buf, S* d_buf, uint32_t pb, uint32_t pe, uint32_t l, uint32_t r,
                       R pivot) -> uint32_t {
      constexpr bool ST = decltype(strict_tag)::value;
      uint32_t base = pb;
      for (; base + U * WAVE <= pe; base += U * WAVE) {
        R kx[U];
        bool isl[U];
        uint64_t ml[U];
#pragma unroll
        for (int u = 0; u < U; u++) kx[u] = (R)s_buf[base + u * WAVE + lane];
#pragma unroll
        for (int u = 0; u < U; u++) {
          isl[u] = ST ? K::lt(kx[u], pivot) : !K::lt(pivot, kx[u]);
          ml[u] = ballot(isl[u]);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          const uint32_t lrank = mbcnt(ml[u]);
          const uint32_t d = isl[u] ? l + lrank : r - 1 - ((uint32_t)lane - lrank);
          d_buf[d] = (S)kx[u];
          const uint32_t nlft = (uint32_t)__popcll(ml[u]);
          l += nlft;
          r -= (uint32_t)WAVE - nlft;
        }
      }
      for (; base < pe; base += WAVE) {
        const uint32_t i = base + lane;
        const bool valid = i < pe;
        const R kx = (R)s_buf[valid ? i : pe - 1];
        const bool isl = valid && (ST ? K::lt(kx, pivot) : !K::lt(pivot, kx));
        const uint64_t ml = ballot(isl), vm = ballot(valid);
        const uint32_t lrank = mbcnt(ml), vrank = mbcnt(vm);
        const uint32_t d = isl ? l + lrank : r - 1 - (vrank - lrank);
        if (valid) d_buf[d] = (S)kx;
        const uint32_t nlft = (uint32_t)__popcll(ml);
        l += nlft;
        r -= (uint32_t)__popcll(vm) - nlft;
      }
      return l;
    };
    // left count of [pb, pe) (the wave groups' counting pass)
    auto count_left = [&](auto strict_tag, const S* s_buf, uint32_t pb, uint32_t pe, R pivot) -> uint32_t {
      constexpr bool ST = decltype(strict_tag)::value;
      uint32_t cnt = 0, base = pb;
      for (; base + U * WAVE <= pe; base += U * WAVE) {
        R kx[U];
#pragma unroll
        for (int u = 0; u < U; u++) kx[u] = (R)s_buf[base + u * WAVE + lane];
#pragma unroll
        for (int u = 0; u < U; u++) cnt += (uint32_t)__popcll(ballot(ST ? K::lt(kx[u], pivot) : !K::lt(pivot, kx[u])));
      }
      for (; base < pe; base += WAVE) {
        const uint32_t i = base + lane;
        const bool valid = i < pe;
        const R kx = (R)s_buf[valid ? i : pe - 1];
        cnt += (uint32_t)__popcll(ballot(valid && (ST ? K::lt(kx, pivot) : !K::lt(pivot, kx))));
      }
      return cnt;
    };
    // The range minimum is needed only when nothing went right (Alg. 1's degenerate
    // case, whose next pivot it is): taken then, from the partition's output, by one wave.
    auto range_min = [&](const S* buf, uint32_t lb, uint32_t le) -> R {
      R m = K::maxv();
      for (uint32_t i = lb + lane; i < le; i += WAVE) m = K::kmin(m, (R)buf[i]);
      return wave_min<K>(m);
    };
    if (G == 1) {
      for (uint32_t it_i = wave; it_i < nitems; it_i += SOLO_NW) {
        LocalItem<K> it = ls.list[cur][it_i];
        if (!admit(it, true)) continue;
        const bool strict = (it.flags & LI_STRICT) != 0;
        S* s_buf = (it.flags & LI_INB) ? bufB : bufA;
        S* d_buf = (it.flags & LI_INB) ? bufA : bufB;
        const R pivot = pick_pivot(it, it_i, s_buf);
        R mn = K::maxv();
        if constexpr (IP) {
          // the in-place scan's order (Sec. 2.1), so that later pivots see the same ranges
          const uint32_t bound = ip_partition_wave<K>(s_buf, d_buf, it.lb, it.le, pivot, strict, mn);
          plan(it, bound, mn, pivot);
        } else {
          const uint32_t bound = strict ? scatter(std::true_type{}, s_buf, d_buf, it.lb, it.le, it.lb, it.le, pivot)
                                        : scatter(std::false_type{}, s_buf, d_buf, it.lb, it.le, it.lb, it.le, pivot);
          if (bound == it.le && !strict) mn = range_min(d_buf, it.lb, it.le);
          plan(it, bound, mn, pivot);
        }
      }
    } else {
      // wave group: wave sw of item wave / G takes the sw-th part of the range; a
      // counting pass gives every part its output positions, so the result is the one
      // a single wave scanning the whole range would write
      const int item = wave / G, sw = wave % G;
      const bool have = (uint32_t)item < nitems;   // waves past the last range only keep step
      LocalItem<K> it = ls.list[cur][have ? item : 0];
      const bool go = have && admit(it, sw == 0);
      const bool strict = (it.flags & LI_STRICT) != 0;
      S* s_buf = (it.flags & LI_INB) ? bufB : bufA;
      S* d_buf = (it.flags & LI_INB) ? bufA : bufB;
      const uint32_t len = it.le - it.lb;
      const uint32_t per = ((len + G - 1) / G + U * WAVE - 1) / (U * WAVE) * (U * WAVE);
      auto part_b = [&](int q) { const uint32_t o = (uint32_t)q * per; return it.lb + (o < len ? o : len); };
      // every wave of the group draws the same pivot itself: no broadcast barrier
      const R pivot = go ? pick_pivot(it, (uint32_t)item, s_buf) : K::maxv();
      if constexpr (IP) {
        // the in-place order; the group's block tables live in the next level's
        // pivot-offset rows, which are written only after this level's partitions
        static_assert(sizeof(ls.pvoff[0]) >= (SOLO_NW / 2) * 512, "in-place group tables");
        uint8_t* tab = reinterpret_cast<uint8_t*>(&ls.pvoff[cur ^ 1][0][0]) + item * 512;
        R mn;
        const uint32_t bound = ip_partition_group<K>(s_buf, d_buf, it.lb, it.le, pivot, strict, G, sw, go, tab, mn);
        if (go && lane == 0) ls.gmin[wave] = mn;
        __syncthreads();
        if (go && sw == 0) {
          R gm = K::maxv();
          for (int q = 0; q < G; q++) gm = K::kmin(gm, ls.gmin[item * G + q]);
          plan(it, bound, gm, pivot);
        }
      } else {
      const uint32_t pb = part_b(sw), pe = part_b(sw + 1);
      if (go) {
        const uint32_t cnt = strict ? count_left(std::true_type{}, s_buf, pb, pe, pivot)
                                    : count_left(std::false_type{}, s_buf, pb, pe, pivot);
        if (lane == 0) ls.gcnt[wave] = cnt;
      }
      __syncthreads();
      uint32_t ltot = 0;
      if (go) {
        uint32_t lbef = 0, rbef = 0;
        for (int q = 0; q < G; q++) {
          const uint32_t c = ls.gcnt[item * G + q];
          if (q < sw) {
            lbef += c;
            rbef += (part_b(q + 1) - part_b(q)) - c;
          }
          ltot += c;
        }
        if (strict) scatter(std::true_type{}, s_buf, d_buf, pb, pe, it.lb + lbef, it.le - rbef, pivot);
        else scatter(std::false_type{}, s_buf, d_buf, pb, pe, it.lb + lbef, it.le - rbef, pivot);
      }
      __syncthreads();   // the whole partition is in d_buf before runs of it are copied
      if (go && sw == 0) {
        const uint32_t bound = it.lb + ltot;
        const R gm = (bound == it.le && !strict) ? range_min(d_buf, it.lb, it.le) : K::maxv();
        plan(it, bound, gm, pivot);
      }
      }
    }
    __syncthreads();
    // the next level's ranges are known: one wave computes their ChoosePivot chunk
    // starts, one range per lane (the random-number chain is serial per range, so
    // this takes the time of one range instead of one per range)
    if (wave == SOLO_NW - 1) {
      const uint32_t nn = ls.nlist[cur ^ 1] < (uint32_t)LIST_CAP ? ls.nlist[cur ^ 1] : (uint32_t)LIST_CAP;
      if ((uint32_t)lane < nn) {
        const LocalItem<K> ni = ls.list[cur ^ 1][lane];
        uint64_t o[9];
        pivot_chunk_starts<K>(b + ni.lb, b + ni.le, p, o);
#pragma unroll
        for (int i = 0; i < 9; i++) ls.pvoff[cur ^ 1][lane][i] = (uint32_t)o[i];
      }
    }
    // 3. base cases, four per wave (one per 16-lane group); they are collected over
    // recursion levels and sorted together once the list could overflow at the next
    // level or no range is left to partition
    const bool last = ls.nlist[cur ^ 1] == 0;
    const bool flush_bc = ls.nbc > (uint32_t)(BC_CAP - 2 * LIST_CAP) || last;
    const uint32_t nbc = flush_bc ? (ls.nbc < BC_CAP ? ls.nbc : BC_CAP) : 0u;
    for (uint32_t q0 = wave * 4; q0 < nbc; q0 += SOLO_NW * 4) {
      const uint32_t qi = q0 + (lane >> 4);
      const int gl = lane & 15;
      uint32_t lb = 0, len = 0, inb = 0, isfb = 0;
      if (qi < nbc) {
        const uint32_t w = ls.bc[qi];
        inb = w & 1u;
        isfb = (w >> 1) & 1u;
        len = ((w >> 2) & 255u) + 1;
        lb = w >> 10;
      }
      if (gl == 0 && qi < nbc && !isfb) atomicAdd(&ls.stat_bc, 1u);
      const S* s_buf = inb ? bufB : bufA;
      R x[16];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const uint32_t pos = (uint32_t)(16 * r + gl);
        x[r] = pos < len ? (R)s_buf[lb + pos] : K::maxv();
      }
      network16x16<K>(x);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const uint32_t pos = (uint32_t)(16 * gl + r);
        if (pos < len) bufA[lb + pos] = (S)x[r];
      }
    }
    // 4. bounded-time sorts of this level (whole workgroup, one range at a time).  Their
    // ranges are disjoint from the base cases', so a wave may start on them while
    // others still sort base cases; the list was complete at the barrier after the
    // partitions.
    const uint32_t nbd = ls.nbounded < LIST_CAP ? ls.nbounded : LIST_CAP;
    if (tid == 0 && nbd) atomicAdd(&p.stats->bounded_lds, (unsigned long long)nbd);
    for (uint32_t f = 0; f < nbd; f++) {
      const LocalItem<K> it = ls.bounded[f];
      S* a = (it.flags & LI_INB) ? bufB : bufA;
      wg_bitonic_lds<K, S>(a + it.lb, it.le - it.lb);
      if (it.flags & LI_INB) {
        for (uint32_t i = it.lb + tid; i < it.le; i += SOLO_P) bufA[i] = bufB[i];
      }
      __syncthreads();
    }
    // a flush before the last level empties the list for the next levels, once every
    // wave has read its length (after the last level nothing more is pushed, and the
    // next local sort starts with an empty list)
    const bool reset_bc = flush_bc && !last;
    if (reset_bc) __syncthreads();
    if (tid == 0) {
      if (reset_bc) ls.nbc = 0;
      ls.nbounded = 0;
      ls.nlist[cur] = 0;
    }
    __syncthreads();
    cur ^= 1;
    if (ls.nlist[cur] == 0) break;
  }
  if (lane == 0) {
    if (w_part) {
      atomicAdd(&ls.stat_part, w_part);
      atomicAdd(&ls.stat_pkeys, w_pkeys);
      atomicMax(&ls.stat_maxd, w_maxd);
    }
    if (w_deg) atomicAdd(&ls.stat_deg, w_deg);
    if (w_eq) atomicAdd(&ls.stat_eq, w_eq);
  }
  __syncthreads();
  // 5. write out
  for (uint32_t i = tid; i < n; i += SOLO_P) {
    S val = bufA[i];
    if (!out_internal && p.mode) val = K::store_t((R)val, p.mode);
    out[b + i] = val;
  }
  if (tid == 0) {
    acc.part += ls.stat_part;
    acc.pkeys += ls.stat_pkeys;
    acc.maxd = ls.stat_maxd > acc.maxd ? ls.stat_maxd : acc.maxd;
    acc.bc += ls.stat_bc;
    acc.deg += ls.stat_deg;
    acc.eq += ls.stat_eq;
    acc.fb += ls.stat_fb;
    acc.fbkeys += ls.stat_fbkeys;
  }
  __syncthreads();
}

// ---- solo kernel: whole ranges per workgroup ------------------------------------------

constexpr int STACK_CAP = 48;

// waves per SIMD the solo kernel is compiled for: four (two 512-thread workgroups per
// CU, which their LDS allows) except for 16-byte keys, whose network needs more
// registers
template <int SIZE>
constexpr int solo_waves() { return SIZE == 16 ? 2 : 4; }

// Fill keys[b, e) of the caller's array with one value (output transform applied).
template <class K>
__device__ void fill_range(const Params& p, uint64_t b, uint64_t e, typename K::R v) {
  using S = typename K::S;
  S* out = (S*)p.keys;
  const S val = K::store_t(v, p.mode);
  for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) out[i] = val;
}

// Merge-path merge of sorted runs a[0, na) and c[0, nc) into o[0, na + nc) by the
// workgroup (ties take a first).
template <class K>
__device__ void wg_merge(const typename K::S* a, uint64_t na, const typename K::S* c, uint64_t nc,
                         typename K::S* out) {
  using R = typename K::R;
  const uint64_t total = na + nc;
  const uint64_t per = (total + blockDim.x - 1) / blockDim.x;
  const uint64_t o0 = per * threadIdx.x;
  if (o0 >= total) return;
  const uint64_t o1 = (o0 + per < total) ? o0 + per : total;
  uint64_t lo = o0 > nc ? o0 - nc : 0, hi = o0 < na ? o0 : na;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (!K::lt((R)c[o0 - mid - 1], (R)a[mid])) lo = mid + 1;
    else hi = mid;
  }
  uint64_t i = lo, j = o0 - lo;
  for (uint64_t o = o0; o < o1; o++) {
    bool take_a;
    if (i >= na) take_a = false;
    else if (j >= nc) take_a = true;
    else take_a = !K::lt((R)c[j], (R)a[i]);
    if (take_a) out[o] = a[i++];
    else out[o] = c[j++];
  }
}

// Bounded-time sort for a range past the fallback mode's own depth limit: sort
// LDS-sized chunks with the bitonic network, then merge runs pairwise through the two
// global buffers; the result goes to the caller's array.  O(n log^2 n) work at most.
// Not counted in the recursion counters: the range was counted when it entered
// fallback mode.  Thread 0 adds the keys its passes read and write to rd and wr.
template <class K>
__device__ void fallback_global(const Params& p, typename K::S* bufA, const Seg& it, unsigned long long& rd,
                                unsigned long long& wr) {
  using R = typename K::R;
  using S = typename K::S;
  const uint64_t b = it.b, e = it.e, n = e - b;
  if (threadIdx.x == 0) {
    atomicAdd(&p.stats->bounded_global, 1ull);
    rd += n;   // chunks in, sorted, out
    wr += n;
  }
  S* X = (S*)((it.flags & SEG_SCRATCH) ? p.scratch : p.keys);
  S* Y = (S*)((it.flags & SEG_SCRATCH) ? p.keys : p.scratch);
  const int tmode = (it.flags & SEG_RAW) ? p.mode : 0;
  const uint64_t C = p.local_cap;
  // 1. chunks: X -> LDS -> sorted -> X (internal form)
  for (uint64_t c0 = b; c0 < e; c0 += C) {
    const uint32_t m = (uint32_t)((c0 + C < e) ? C : e - c0);
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      S s = X[c0 + i];
      bufA[i] = tmode ? (S)K::load_t(s, tmode) : s;
    }
    __syncthreads();
    wg_bitonic_lds<K, S>(bufA, m);
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) X[c0 + i] = bufA[i];
    __syncthreads();
  }
  // 2. merge passes
  S* from = X;
  S* to = Y;
  for (uint64_t w = C; w < n; w *= 2) {
    if (threadIdx.x == 0) {
      rd += n;
      wr += n;
    }
    for (uint64_t s = 0; s < n; s += 2 * w) {
      const uint64_t na = (s + w < n) ? w : n - s;
      const uint64_t nc = (s + 2 * w < n) ? w : (s + w < n ? n - s - w : 0);
      wg_merge<K>(from + b + s, na, from + b + s + na, nc, to + b + s);
    }
    __syncthreads();
    S* t = from;
    from = to;
    to = t;
  }
  // 3. output transform into the caller's array
  S* out = (S*)p.keys;
  if (from != out || p.mode != 0) {
    if (threadIdx.x == 0) {
      rd += n;
      wr += n;
    }
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      S v = from[i];
      out[i] = p.mode ? K::store_t((R)v, p.mode) : v;
    }
  }
  __syncthreads();
}

// IP: in-place mode (its own instantiation, so that the default one's registers are
// allocated as without it)
template <class K, bool IP>
__global__ void __launch_bounds__(SOLO_P) __attribute__((amdgpu_waves_per_eu(solo_waves<K::SIZE>()))) solo_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr int SI = solo_chunks(8 * K::SIZE);
  using TL = Tile<K, SOLO_P, SI>;
  constexpr int T = TL::T;
  static_assert(T * sizeof(S) <= LOCAL_BYTES, "tile staging must fit one LDS buffer");
  __shared__ __attribute__((aligned(16))) char lds_raw[2 * LOCAL_BYTES];
  __shared__ LocalShared<K> ls;
  __shared__ typename TL::Aux aux;
  __shared__ Seg stack[STACK_CAP];
  __shared__ int sp;
  __shared__ unsigned long long sh_item;
  __shared__ R sh_min;
  S* bufA = (S*)lds_raw;
  S* bufB = (S*)(lds_raw + LOCAL_BYTES);
  const int tid = threadIdx.x;
  const unsigned long long count = p.solo_ctr->count;
  const unsigned long long nitems = count < p.cap_solo ? count : p.cap_solo;
  unsigned long long hrd = 0, hwr = 0;   // thread 0: keys read / written by whole-key sweeps
  __shared__ LocalCounts acc;            // the local sorts' recursion counts (thread 0 writes)
  if (tid == 0) acc = LocalCounts{};
  for (;;) {
    if (tid == 0) sh_item = atomicAdd(&p.solo_ctr->ticket, 1ull);
    __syncthreads();
    const unsigned long long ii = sh_item;
    if (ii >= nitems) break;
    const Seg item = p.solo[p.solo_order[ii]];
    if (item.flags & SEG_FILL) {
      fill_range<K>(p, item.b, item.e, K::from_u64x2(item.pv_lo, item.pv_hi));
      if (tid == 0) hwr += item.e - item.b;
      __syncthreads();
      continue;
    }
    if (tid == 0) {
      stack[0] = item;
      sp = 1;
    }
    __syncthreads();
    while (sp > 0) {
      Seg cur = stack[sp - 1];
      __syncthreads();
      if (tid == 0) sp--;
      const uint64_t n = cur.e - cur.b;
      const bool in_scratch = (cur.flags & SEG_SCRATCH) != 0;
      const S* src = (const S*)(in_scratch ? p.scratch : p.keys);
      S* dst = (S*)(in_scratch ? p.keys : p.scratch);
      const bool raw = (cur.flags & SEG_RAW) != 0;
      // the bounded-time sort: through the key scratch, or in place without one
      auto bounded = [&](const Seg& sgb) {
        if constexpr (IP) fallback_global_inplace<K>(p, bufA, sgb, hrd, hwr);
        else fallback_global<K>(p, bufA, sgb, hrd, hwr);
        __syncthreads();
      };
      if (cur.flags & SEG_BOUNDED) {
        bounded(cur);
        continue;
      }
      if (n <= p.local_cap) {
        const uint32_t lf = ((cur.flags & SEG_OVERRIDE) ? LI_OVERRIDE : 0u) |
                            ((cur.flags & SEG_FALLBACK) ? LI_FB : 0u) | ((cur.flags & SEG_STRICT) ? LI_STRICT : 0u);
        local_sort<K, IP>(p, ls, bufA, bufB, src, raw, cur.b, cur.e, cur.depth, cur.limit, lf,
                      K::from_u64x2(cur.pv_lo, cur.pv_hi), (S*)p.keys, false, acc);
        if (tid == 0) {
          hrd += n;
          hwr += n;
        }
        continue;
      }
      if (cur.depth > cur.limit) {
        if (cur.flags & SEG_FALLBACK) {
          bounded(cur);
          continue;
        }
        // the paper's depth limit: continue this range in fallback mode
        if (tid == 0) {
          atomicAdd(&p.stats->fallbacks, 1ull);
          atomicAdd(&p.stats->fallback_keys, (unsigned long long)n);
        }
        cur.flags = (cur.flags & (SEG_SCRATCH | SEG_RAW)) | SEG_FALLBACK;
        cur.depth = 1;
        cur.limit = fb_limit_of(p, n);
        if (cur.depth > cur.limit) {   // a fallback-mode limit of 0
          bounded(cur);
          continue;
        }
      }
      const bool fb = (cur.flags & SEG_FALLBACK) != 0;
      const bool strict = (cur.flags & SEG_STRICT) != 0;
      // pivot
      if (cur.flags & SEG_OVERRIDE) {
        if (tid == 0) aux.pivot = K::from_u64x2(cur.pv_lo, cur.pv_hi);
      } else if (tid < WAVE) {
        const S* sb = src + cur.b;
        const int tm = raw ? p.mode : 0;
        R pv = choose_pivot_wave<K>(
            [&](uint64_t i) -> R {
              S s = sb[i];
              R r;
              if constexpr (sizeof(S) == sizeof(R)) r = s; else r = (R)s;
              return tm ? K::load_t(s, tm) : r;
            },
            cur.b, cur.e, p);
        if (tid == 0) aux.pivot = pv;
      }
      __syncthreads();
      const R pivot = aux.pivot;
      if (IP && n > IP_SOLO_MAX) {   // (ranges are routed here only up to the threshold)
        if (tid == 0) set_err(p, ERR_SOLO_OVERFLOW);
        __syncthreads();
        continue;
      }
      R mn = K::maxv();
      uint64_t bound;
      if constexpr (IP) {
        // in place, in the paper's bidirectional order (a counting pass, then the pass
        // that moves the keys)
        bound = ip_partition_workgroup<K, SOLO_P>((S*)p.keys, cur.b, cur.e, pivot, strict, raw ? p.mode : 0, bufA,
                                                  bufB, &mn);
        if (tid == 0) hrd += n;
      } else {
      // partition tile by tile: src -> dst
      const S* src_aligned = src - p.off;
      const uint64_t k0 = (cur.b + p.off) / T, k1 = (cur.e - 1 + p.off) / T;
      uint64_t excl_l = 0, excl_r = 0;
      for (uint64_t k = k0; k <= k1; k++) {
        const uint64_t vs = (k * T > cur.b + p.off) ? k * T : cur.b + p.off;
        const uint64_t ve = ((k + 1) * T < cur.e + p.off) ? (k + 1) * T : cur.e + p.off;
        R key[SI][K::V];
        TL::template load<false>(src_aligned, k, vs, ve, raw ? p.mode : 0, key);
        R tmin;
        const uint32_t nl = TL::rank_and_stage(bufA, aux, key, k, vs, ve, pivot, strict, &tmin, [](uint32_t, R) {});
        const uint32_t nvalid = (uint32_t)(ve - vs);
        const uint32_t nr = nvalid - nl;
        TL::write_out_keys(bufA, dst, nl, nvalid, cur.b + excl_l, cur.e - excl_r - nr, 0, p.n_total);
        excl_l += nl;
        excl_r += nr;
        if (tid == 0) mn = K::kmin(mn, tmin);
        __syncthreads();
      }
      bound = cur.b + excl_l;
      }
      if (tid == 0) {
        sh_min = mn;
        hrd += n;
        hwr += n;
        if (!fb) {
          acc.gpart++;
          acc.gkeys += n;
          acc.maxd = cur.depth > acc.maxd ? cur.depth : acc.maxd;
        } else {
          acc.fbpart++;
        }
      }
      __syncthreads();
      const uint32_t cf = (in_scratch || IP ? 0u : SEG_SCRATCH) | (fb ? SEG_FALLBACK : 0u);
      // keys of [fb_, fe_) equal the pivot and are final.  Whole range: the caller's
      // array holds the range's keys (source or partition output), so only transformed
      // keys need writing back; part of a range: unless the partition wrote the
      // caller's array untransformed, it holds other keys there.  In place: the
      // partition wrote the caller's array in internal form
      auto retire_equal = [&](uint64_t fb_, uint64_t fe_, bool part) {
        const bool need = IP ? p.mode != 0 : part ? (!in_scratch || p.mode != 0) : (p.mode != 0 && !raw);
        if (need && fe_ > fb_) {
          fill_range<K>(p, fb_, fe_, pivot);
          if (tid == 0) hwr += fe_ - fb_;
        }
      };
      auto push = [&](const Seg& sgn) {
        if (sgn.e <= sgn.b) return;
        if (sp < STACK_CAP) stack[sp++] = sgn;
        else set_err(p, ERR_STACK);
      };
      if (strict) {
        retire_equal(bound, cur.e, true);
        if (tid == 0) push(make_seg<K>(cur.b, bound, cur.depth + 1, cur.limit, cf, pivot));
      } else if (bound == cur.e && !fb) {
        const R segmin = sh_min;
        if (tid == 0) atomicAdd(&p.stats->degenerate, 1ull);
        if (K::eq(segmin, pivot)) {
          if (tid == 0) atomicAdd(&p.stats->all_equal, 1ull);
          retire_equal(cur.b, cur.e, false);
        } else if (tid == 0) {
          push(make_seg<K>(cur.b, cur.e, cur.depth + 1, cur.limit, cf | SEG_OVERRIDE, segmin));
        }
      } else if (bound == cur.e) {
        if (tid == 0) push(make_seg<K>(cur.b, cur.e, cur.depth + 1, cur.limit, cf | SEG_OVERRIDE | SEG_STRICT, pivot));
      } else if (tid == 0) {
        // larger first, so the smaller range is taken next (stack depth <= log2 n)
        const bool left_small = (bound - cur.b) <= (cur.e - bound);
        const Seg l = make_seg<K>(cur.b, bound, cur.depth + 1, cur.limit, cf, pivot);
        const Seg r = make_seg<K>(bound, cur.e, cur.depth + 1, cur.limit, cf, pivot);
        if (left_small) {
          push(r);
          push(l);
        } else {
          push(l);
          push(r);
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0 && (hrd | hwr)) {
    atomicAdd(&p.stats->hbm_read_keys, hrd);
    atomicAdd(&p.stats->hbm_write_keys, hwr);
  }
  if (tid == 0) {
    if (acc.part | acc.gpart) {
      atomicAdd(&p.stats->partitions, acc.part + acc.gpart);
      atomicAdd(&p.stats->keys_partitioned, acc.pkeys + acc.gkeys);
      atomicMax(&p.stats->max_depth, acc.maxd);
    }
    if (acc.part) atomicAdd(&p.stats->lds_partitions, acc.part);
    if (acc.gpart) atomicAdd(&p.stats->global_solo_partitions, acc.gpart);
    if (acc.fbpart) atomicAdd(&p.stats->fallback_partitions, acc.fbpart);
    if (acc.bc) atomicAdd(&p.stats->basecases, acc.bc);
    if (acc.deg) atomicAdd(&p.stats->degenerate, acc.deg);
    if (acc.eq) atomicAdd(&p.stats->all_equal, acc.eq);
    if (acc.fb) {
      atomicAdd(&p.stats->fallbacks, acc.fb);
      atomicAdd(&p.stats->fallback_keys, acc.fbkeys);
    }
  }
}

// The solo list's order of service, before the solo launch: ranges longer than half
// the solo threshold first, then the shorter ones and the fills.  Workgroups take items
// one by one, so the last items taken should be short: a long range taken last holds
// its workgroup while the others have nothing left.  (Order within each class: that of
// the wave-aggregated reservations.)
constexpr int ORDER_P = 256;
template <class K>
__global__ void __launch_bounds__(ORDER_P) solo_order_kernel(Params p) {
  const unsigned long long count = p.solo_ctr->count;
  const uint64_t nitems = count < p.cap_solo ? count : p.cap_solo;
  const int lane = lane_id();
  for (uint64_t base = (uint64_t)blockIdx.x * ORDER_P + (threadIdx.x & ~(WAVE - 1)); base < nitems;
       base += (uint64_t)gridDim.x * ORDER_P) {
    const uint64_t i = base + lane;
    const bool valid = i < nitems;
    bool big = false;
    if (valid) {
      const Seg& s = p.solo[i];
      big = !(s.flags & SEG_FILL) && (s.e - s.b) > p.solo_max / 2;
    }
    const uint64_t mb = ballot(valid && big), ms = ballot(valid && !big);
    unsigned long long b0 = 0, s0 = 0;
    if (lane == 0) {
      if (mb) b0 = atomicAdd(&p.solo_ctr->big, (unsigned long long)__popcll(mb));
      if (ms) s0 = atomicAdd(&p.solo_ctr->small, (unsigned long long)__popcll(ms));
    }
    b0 = __shfl(b0, 0);
    s0 = __shfl(s0, 0);
    if (valid) {
      const uint64_t pos = big ? b0 + mbcnt(mb) : nitems - 1 - (s0 + mbcnt(ms));
      p.solo_order[pos] = (uint32_t)i;
    }
  }
}

// ---- setup ----------------------------------------------------------------------------------

// Clear counters, statistics and look-back words.
template <class K>
__global__ void clear_kernel(Params p) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gid; i < p.cap_tiles; i += stride) p.flags[i] = 0;
  for (uint64_t i = gid; i < (uint64_t)p.max_levels; i += stride) {
    p.lvl_ctr[i].packed = 0;
    p.lvl_ctr[i].keys = 0;
    p.lvl_ctr[i].ticket = 0;
    p.lvl_ctr[i].ticket2 = 0;
    p.lvl_ctr[i].pad2 = 0;
  }
  if (gid == 0) {
    p.solo_ctr->count = 0;
    p.solo_ctr->ticket = 0;
    p.solo_ctr->big = 0;
    p.solo_ctr->small = 0;
    *p.err = 0;
    unsigned long long* st = (unsigned long long*)p.stats;
    for (size_t i = 0; i < sizeof(DevStats) / 8; i++) st[i] = 0;
  }
}

// Route the input ranges: offsets (nseg + 1 entries), or [0, n) when offsets is null.
template <class K>
__global__ void seed_kernel(Params p, const int64_t* offsets, uint64_t nseg) {
  using TL = Tile<K, LEVEL_P, K::LI>;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gid; i < nseg; i += stride) {
    const uint64_t b = offsets ? (uint64_t)offsets[i] : 0;
    const uint64_t e = offsets ? (uint64_t)offsets[i + 1] : p.n_total;
    if (e <= b) continue;
    Seg s{};
    s.b = b;
    s.e = e;
    s.depth = 1;
    s.limit = p.fixed_limit >= 0 ? (uint32_t)p.fixed_limit : depth_limit_of(e - b);
    s.flags = p.seed_level ? SEG_SCRATCH : SEG_RAW;
    route<K, TL::T>(p, s, p.seed_level);
  }
}

}  // namespace vqs
