// vqs_inplace.h -- in-place partitions (Sec. 2.1: the bidirectional scan with
// CompressStore), for the device-wide levels, the solo kernel's global partitions and
// the local sort in LDS.  Included by vqs_kernels.h.
//
// The order they produce is that of the paper's sequential scan with a vector of 64
// keys (one wavefront) and four vectors per loop iteration (a 256-key block):
//
//  * the remainder (len mod 256 keys at the range start; every key when the range has
//    fewer than two blocks) is split first: its left keys go to the range start in
//    order, its right keys to the range end in order, and the range's last keys (as
//    many) take the place between them;
//  * of the remaining whole blocks the first and the last are held back; the loop then
//    reads one block per iteration from the side with the smaller capacity (distance
//    between read and write position; the left side on a tie) and stores each vector
//    in address order: left keys at writeL, right keys just below writeR (which moves
//    down by their number), both in lane order;
//  * the held-back blocks are stored last, first then last.
//
// Parallel form.  After i blocks read on the left and j on the right, the left
// capacity minus the right one is 2 * (256 i - left keys read so far), so the loop
// reads on the left exactly when A(i) <= B(j), with A(i) the right keys among the
// first i loop blocks and B(j) the left keys among the last j.  Both are
// non-decreasing: the read order is the merge of A and B (ties to A), and a block's
// iteration is its rank in that merge.  Counts per block (one pass) therefore give
// every block its iteration and its output offsets.  Every store of an iteration lands
// on keys read at or before it (the capacity invariant), and the remainder and the
// held-back blocks are read before any store: so a tile that takes iterations in order
// only waits until every earlier tile of its range has read its keys.
#pragma once
// (included inside namespace vqs)

static_assert(IP_V == WAVE, "an in-place vector is one wavefront");

template <class K>
__device__ inline typename K::R ip_load(const typename K::S* a, uint64_t i, int tmode) {
  const typename K::S s = a[i];
  typename K::R r;
  if constexpr (sizeof(typename K::S) == sizeof(typename K::R)) {
    r = s;
  } else {
    r = (typename K::R)s;
  }
  return tmode ? K::load_t(s, tmode) : r;
}

template <class K>
__device__ inline typename K::S ip_s(typename K::R r) {
  if constexpr (sizeof(typename K::S) == sizeof(typename K::R)) {
    return r;
  } else {
    return (typename K::S)r;
  }
}

// the partition predicate: left = not after the pivot (strict: before it)
template <class K>
__device__ inline bool ip_left(typename K::R x, typename K::R pv, bool strict) {
  return strict ? K::lt(x, pv) : !K::lt(pv, x);
}

constexpr unsigned long long IP_ST_AGG = 1ull << 46, IP_ST_INC = 2ull << 46, IP_VAL = (1ull << 46) - 1;
// predecessors an in-place look-back step polls: the nearest inclusive tile is usually
// a few tiles back, and polling 64 device-coherent words per step cost 3 % (1e8 u64)
constexpr int IP_LB_WIN = 16;

// Decoupled look-back over the tiles [g0, g) of a range, one wave: waits until every
// predecessor back to the nearest inclusive one has published in this epoch and returns
// the sum of their values (so afterwards every earlier tile of the range has
// published).  Device-coherent single-word accesses only.  A spin limit, or an error
// raised elsewhere, ends the wait with ERR_SPIN.
__device__ inline unsigned long long ip_lookback(const Params& p, unsigned long long g, unsigned long long g0,
                                                 unsigned long long epoch) {
  const int lane = lane_id();
  unsigned long long excl = 0;
  if (g == g0) return 0;
  unsigned long long top = g - 1;
  uint32_t spins = 0;
  for (;;) {
    const bool inr = lane < IP_LB_WIN && top >= g0 + (unsigned long long)lane;
    unsigned long long f = 0;
    if (inr) f = __hip_atomic_load(&p.flags[top - lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ready = inr && (f & ~((1ull << 48) - 1)) == epoch && (f & (3ull << 46)) != 0;
    const bool inc = ready && (f & IP_ST_INC);
    const uint64_t incm = ballot(inc), readym = ballot(ready), inrm = ballot(inr);
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
    unsigned long long v = (((need >> lane) & 1ull) != 0) ? (f & IP_VAL) : 0ull;
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) v += (unsigned long long)__shfl_xor((long long)v, m);
    excl += v;
    if (incm) break;
    if (top < g0 + IP_LB_WIN) break;   // cannot happen: tile g0 always publishes inclusive
    top -= IP_LB_WIN;
  }
  return excl;
}

__device__ inline void ip_publish(const Params& p, unsigned long long g, unsigned long long word) {
  __hip_atomic_store(&p.flags[g], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stores of one vector (the whole wave, lane order): left keys from wl, right keys
// ending at wr_end (exclusive); returns the vector's left count.
template <class K, class Store>
__device__ inline uint32_t ip_store_vector(typename K::R x, bool left, Store&& store, uint64_t wl, uint64_t wr_end) {
  const int lane = lane_id();
  const uint64_t ml = ballot(left);
  const uint32_t lr = mbcnt(ml), nlv = (uint32_t)__popcll(ml);
  if (left) store(wl + lr, x);
  else store(wr_end - (IP_V - nlv) + ((uint32_t)lane - lr), x);
  return nlv;
}

// The held-back blocks (saved keys sv[0, 2 * IP_B): first block, then last) of a range
// whose loop wrote lc left and rc right keys: stored by waves 0 (first block) and 1
// (last block; cfirst = the first block's left count) from ms + lc and below me - rc.
template <class K, class Load, class Store>
__device__ inline void ip_store_held(Load&& sv, Store&& store, uint64_t ms, uint64_t me, uint64_t lc, uint64_t rc,
                                     uint32_t cfirst, typename K::R pv, bool strict, int wave) {
  if (wave > 1) return;
  const int lane = lane_id();
  uint64_t l = lc + (wave ? cfirst : 0u);
  uint64_t r = rc + (wave ? (uint64_t)(IP_B - cfirst) : 0u);
#pragma unroll
  for (int v = 0; v < IP_U; v++) {
    const typename K::R x = sv((uint32_t)(wave * IP_B + v * IP_V + lane));
    const uint32_t nlv = ip_store_vector<K>(x, ip_left<K>(x, pv, strict), store, ms + l, me - r);
    l += nlv;
    r += IP_V - nlv;
  }
}

// The remainder (saved keys sv[0, nrem)): left keys from b in order, right keys from
// me in order (one wave).
template <class K, class Load, class Store>
__device__ inline void ip_store_remainder(Load&& sv, Store&& store, uint64_t b, uint64_t me, uint32_t nrem,
                                          typename K::R pv, bool strict) {
  const int lane = lane_id();
  uint32_t l = 0, r = 0;
  for (uint32_t x0 = 0; x0 < nrem; x0 += WAVE) {
    const bool valid = x0 + (uint32_t)lane < nrem;
    const typename K::R x = sv(valid ? x0 + (uint32_t)lane : 0u);
    const bool left = valid && ip_left<K>(x, pv, strict);
    const uint64_t ml = ballot(left), mr = ballot(valid && !left);
    if (left) store(b + l + mbcnt(ml), x);
    else if (valid) store(me + r + mbcnt(mr), x);
    l += (uint32_t)__popcll(ml);
    r += (uint32_t)__popcll(mr);
  }
}

// ---- device-wide in-place levels ---------------------------------------------------------
//
// A level's ranges (all longer than the solo threshold) are cut into tiles of
// ip_steps loop iterations.  ip_count_kernel: every tile counts the left keys of its
// loop blocks (in address order) and a look-back gives their prefix over the range;
// tile 0 also saves the remainder and the held-back blocks.  ip_scatter_kernel: tile t
// takes iterations [t * steps, (t + 1) * steps): a merge-path search on the prefix
// finds the blocks it reads, it loads and stages them, waits (look-back) until every
// earlier tile of the range has loaded, then writes its two contiguous runs.  Tile 0
// writes the remainder, the last tile the held-back blocks, and plans the children.

// A level's ranges, one wave each, after their pivots are known: the remainder's left
// count, the remainder and the held-back blocks saved in internal form (the partition
// launch overwrites their places before it stores them), the held-back blocks' left
// counts, the smallest of these keys, and every tile's range.
constexpr int IP_PRO_P = 256;

template <class K>
__global__ void __launch_bounds__(IP_PRO_P) ip_prologue_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr uint32_t ST = ip_steps_of(K::SIZE);
  const int L = p.level;
  const uint32_t nseg = (uint32_t)(p.lvl_ctr[L].packed >> 40);
  const Seg* segs = p.lvl_segs[L & 1];
  const unsigned long long* tbase = p.lvl_tbase[L & 1];
  const S* keys = (const S*)p.keys;
  const int tmode = (L == 0) ? p.mode : 0;
  const int lane = lane_id();
  const uint32_t wave0 = (blockIdx.x * IP_PRO_P + threadIdx.x) / WAVE;
  const uint32_t nwaves = gridDim.x * (IP_PRO_P / WAVE);
  unsigned long long keys_read = 0;
  for (uint32_t si = wave0; si < nseg; si += nwaves) {
    const Seg sg = segs[si];
    if (lane == 0 && !(sg.flags & (SEG_PIVOT | SEG_OVERRIDE))) set_err(p, ERR_NO_PIVOT);
    const uint64_t len = sg.e - sg.b;
    const uint32_t nrem = (uint32_t)(len % IP_B);
    const uint64_t nt = ip_tiles_of(len, ST);
    const R pv = K::from_u64x2(sg.pv_lo, sg.pv_hi);
    const bool strict = (sg.flags & SEG_STRICT) != 0;
    S* sv = (S*)p.ip_stash + (uint64_t)si * IP_STASH;
    R mn = K::maxv();
    // the remainder (at most four vectors, all loads first)
    R rk[IP_U];
#pragma unroll
    for (int u = 0; u < IP_U; u++) {
      const uint32_t i = (uint32_t)(u * IP_V + lane);
      rk[u] = ip_load<K>(keys, sg.b + (i < nrem ? i : 0u), tmode);
    }
    uint32_t lrem = 0;
#pragma unroll
    for (int u = 0; u < IP_U; u++) {
      const uint32_t i = (uint32_t)(u * IP_V + lane);
      if (i < nrem) {
        sv[i] = ip_s<K>(rk[u]);
        mn = K::kmin(mn, rk[u]);
      }
      lrem += (uint32_t)__popcll(ballot(i < nrem && ip_left<K>(rk[u], pv, strict)));
    }
    const uint32_t rrem = nrem - lrem;
    const uint64_t ms = sg.b + lrem, me = sg.e - rrem;
    // the held-back blocks: main index y of the first block is the range's last rrem
    // keys, then the keys after the remainder's left ones
    R hk[2 * IP_U];
#pragma unroll
    for (int u = 0; u < 2 * IP_U; u++) {
      const uint32_t y = (uint32_t)((u % IP_U) * IP_V + lane);
      hk[u] = ip_load<K>(keys, u < IP_U ? (y < rrem ? me + y : ms + y) : me - IP_B + y, tmode);
    }
    uint32_t cf = 0, cl = 0;
#pragma unroll
    for (int u = 0; u < 2 * IP_U; u++) {
      sv[IP_B + u * IP_V + lane] = ip_s<K>(hk[u]);
      mn = K::kmin(mn, hk[u]);
      const uint32_t c = (uint32_t)__popcll(ballot(ip_left<K>(hk[u], pv, strict)));
      if (u < IP_U) cf += c;
      else cl += c;
    }
    mn = wave_min<K>(mn);
    if (lane == 0) {
      IpRange r{lrem, cf, cl, 0u, 0, 0};
      to_words<K>(mn, r.mn_lo, r.mn_hi);
      p.ip_rng[si] = r;
    }
    const unsigned long long g0 = tbase[si];
    for (uint64_t t = (uint64_t)lane; t < nt; t += WAVE) p.ip_tseg[g0 + t] = si;
    keys_read += nrem + 2 * IP_B;
  }
  if (lane == 0 && keys_read) atomicAdd(&p.stats->hbm_read_keys, keys_read);
}

// (four waves per SIMD: in place 2.5e8 f32 -7 %, 2e8 u16 -13 %)
template <class K>
__global__ void __launch_bounds__(LEVEL_P) __attribute__((amdgpu_waves_per_eu(4))) ip_count_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr uint32_t ST = ip_steps_of(K::SIZE);
  constexpr int NW = LEVEL_P / WAVE;
  static_assert(ST <= WAVE, "one lane per block of a tile");
  __shared__ unsigned long long sh_ticket, sh_excl;
  __shared__ uint32_t sh_cnt[ST];   // loop blocks of the tile
  __shared__ R sh_wmin[NW];

  const int L = p.level;
  const unsigned long long packed = p.lvl_ctr[L].packed;
  const unsigned long long ntiles = packed & TILE_MASK40;
  if (ntiles == 0) return;
  const Seg* segs = p.lvl_segs[L & 1];
  const unsigned long long* tbase = p.lvl_tbase[L & 1];
  const S* keys = (const S*)p.keys;
  const int tmode = (L == 0) ? p.mode : 0;
  const unsigned long long epoch = (unsigned long long)(2 * L + 1) << 48;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
  unsigned long long keys_read = 0;
  for (;;) {
    if (tid == 0) sh_ticket = atomicAdd(&p.lvl_ctr[L].ticket, 1u);
    __syncthreads();
    const unsigned long long g = sh_ticket;
    if (g >= ntiles) break;
    const uint32_t si = p.ip_tseg[g];
    const Seg sg = segs[si];
    const unsigned long long g0 = tbase[si];
    const uint64_t t = g - g0;
    const uint64_t len = sg.e - sg.b;
    const uint64_t nl = ip_loop_blocks(len);
    const R pv = K::from_u64x2(sg.pv_lo, sg.pv_hi);
    const bool strict = (sg.flags & SEG_STRICT) != 0;
    // the remainder's left count (from the prologue) places the loop blocks
    const uint64_t ms = sg.b + p.ip_rng[si].lrem;
    const uint64_t k0 = 1 + t * ST;   // the tile's first loop block
    const uint32_t nblk = t * ST < nl ? (uint32_t)(nl - t * ST < ST ? nl - t * ST : ST) : 0u;
    R mn = K::maxv();
    {
      // wave w counts blocks w, w + NW, ...: all of its loads issued before any is used
      constexpr int BPW = (int)((ST + NW - 1) / NW);
      R x[BPW][IP_U];
#pragma unroll
      for (int r = 0; r < BPW; r++) {
        const uint32_t kk = (uint32_t)w + (uint32_t)r * NW;
#pragma unroll
        for (int v = 0; v < IP_U; v++)
          x[r][v] = ip_load<K>(keys, kk < nblk ? ms + (k0 + kk) * IP_B + v * IP_V + lane : sg.b, tmode);
      }
#pragma unroll
      for (int r = 0; r < BPW; r++) {
        const uint32_t kk = (uint32_t)w + (uint32_t)r * NW;
        if (kk < nblk) {
          uint32_t c = 0;
#pragma unroll
          for (int v = 0; v < IP_U; v++) {
            mn = K::kmin(mn, x[r][v]);
            c += (uint32_t)__popcll(ballot(ip_left<K>(x[r][v], pv, strict)));
          }
          if (lane == 0) sh_cnt[kk] = c;
        }
      }
    }
    mn = wave_min<K>(mn);
    if (lane == 0) sh_wmin[w] = mn;
    __syncthreads();
    uint32_t tot = 0;
    for (uint32_t k = 0; k < nblk; k++) tot += sh_cnt[k];
    if (tid == 0) {
      R m2 = sh_wmin[0];
#pragma unroll
      for (int ww = 1; ww < NW; ww++) m2 = K::kmin(m2, sh_wmin[ww]);
      uint64_t lo, hi;
      to_words<K>(m2, lo, hi);
      p.tilemin[g].lo = lo;   // read by the partition launch
      p.tilemin[g].hi = hi;
      if (t != 0) ip_publish(p, g, epoch | IP_ST_AGG | tot);
    }
    if (w == 0) {
      const unsigned long long excl = ip_lookback(p, g, g0, epoch);
      if (lane == 0) {
        ip_publish(p, g, epoch | IP_ST_INC | (excl + tot));
        sh_excl = excl;
      }
    }
    __syncthreads();
    if (w == 0) {
      uint64_t v = (uint32_t)lane < nblk ? sh_cnt[lane] : 0u;
      v = wave_incl_scan64(v);
      if ((uint32_t)lane < nblk) p.ip_pfx[g0 * ST + (k0 - 1) + lane] = sh_excl + v;
    }
    if (tid == 0) keys_read += (uint64_t)nblk * IP_B;
    __syncthreads();
  }
  if (tid == 0 && keys_read) atomicAdd(&p.stats->hbm_read_keys, keys_read);
}

template <class K>
__global__ void __launch_bounds__(LEVEL_P) __attribute__((amdgpu_waves_per_eu(4))) ip_scatter_kernel(Params p) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr uint32_t ST = ip_steps_of(K::SIZE);
  constexpr uint32_t NV = ST * IP_U;   // vectors per tile
  constexpr int NW = LEVEL_P / WAVE;
  constexpr int VPW = (int)((NV + NW - 1) / NW);
  constexpr int VPL = (int)((NV + WAVE - 1) / WAVE);   // vectors per lane of the scan
  using TW = Tile<K, LEVEL_P, 1>;
  __shared__ __attribute__((aligned(16))) S stage[ST * IP_B];
  __shared__ unsigned long long sh_ticket, sh_lc0, sh_fill0;
  __shared__ uint32_t sh_nlt;
  __shared__ uint32_t sh_blk[ST];
  __shared__ uint32_t sh_vc[NV], sh_vlo[NV], sh_vro[NV];
  __shared__ R sh_wmin[NW];
  __shared__ R sh_segmin;

  const int L = p.level;
  const unsigned long long packed = p.lvl_ctr[L].packed;
  const unsigned long long ntiles = packed & TILE_MASK40;
  if (ntiles == 0) return;
  const Seg* segs = p.lvl_segs[L & 1];
  const unsigned long long* tbase = p.lvl_tbase[L & 1];
  S* keys = (S*)p.keys;
  const int tmode = (L == 0) ? p.mode : 0;
  const unsigned long long epoch = (unsigned long long)(2 * L + 2) << 48;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
  unsigned long long tiles_done = 0, nread = 0, nwritten = 0;
  auto store_key = [&](uint64_t i, R x) { keys[i] = ip_s<K>(x); };
  for (;;) {
    // tiles are taken in ticket order (the look-back waits only on earlier tickets)
    if (tid == 0) sh_ticket = atomicAdd(&p.lvl_ctr[L].ticket2, 1u);
    __syncthreads();
    const unsigned long long g = sh_ticket;
    if (g >= ntiles) break;
    const uint32_t si = p.ip_tseg[g];
    const Seg sg = segs[si];
    const unsigned long long g0 = tbase[si];
    const uint64_t t = g - g0;
    const uint64_t len = sg.e - sg.b;
    const uint32_t nrem = (uint32_t)(len % IP_B);
    const uint64_t nl = ip_loop_blocks(len);
    const uint64_t nt = ip_tiles_of(len, ST);
    const R pv = K::from_u64x2(sg.pv_lo, sg.pv_hi);
    const bool strict = (sg.flags & SEG_STRICT) != 0;
    const IpRange ir = p.ip_rng[si];
    const uint32_t lrem = ir.lrem, rrem = nrem - lrem;
    const uint64_t ms = sg.b + lrem, me = sg.e - rrem;
    const unsigned long long* pf = p.ip_pfx + g0 * ST;   // pf[k - 1]: left keys of loop blocks 1..k
    const uint64_t s0 = t * ST;
    const uint32_t ns = s0 < nl ? (uint32_t)(nl - s0 < ST ? nl - s0 : ST) : 0u;
    // 1. the tile's iterations: blocks read, and the left keys stored before the first
    if (w == 0) {
      const uint64_t Q = nl ? pf[nl - 1] : 0;
      auto Pv = [&](uint64_t k) -> uint64_t { return k ? pf[k - 1] : 0ull; };
      auto A = [&](uint64_t i) -> uint64_t { return (uint64_t)IP_B * i - Pv(i); };
      auto B = [&](uint64_t j) -> uint64_t { return Q - Pv(nl - j); };
      // blocks read on the left before iteration s0: the first i in [0, s0] with
      // i == s0 or A(i) > B(s0 - 1 - i) (the merge path through the diagonal s0)
      uint64_t lo = 0, hi = s0;
      while (lo < hi) {
        const uint64_t span = hi - lo;
        const uint64_t step = (span + WAVE - 1) / WAVE;
        const uint64_t c = lo + (uint64_t)lane * step;
        const bool f = c >= hi || A(c) > B(s0 - 1 - c);
        const uint64_t fm = ballot(f);
        if (fm == 0) {
          lo = lo + (uint64_t)(WAVE - 1) * step + 1;
        } else {
          const int fl = __builtin_ctzll(fm);
          const uint64_t cf = lo + (uint64_t)fl * step;
          if (fl > 0) lo = lo + (uint64_t)(fl - 1) * step + 1;
          hi = cf < hi ? cf : hi;
        }
      }
      const uint64_t i0 = lo, j0 = s0 - lo;
      uint64_t aw = 0, bw = 0;
      if (ns) {
        aw = i0 + lane < nl ? A(i0 + lane) : ~0ull;
        bw = j0 + lane < nl ? B(j0 + lane) : ~0ull;
      }
      const uint64_t a0 = read_lane(aw, 0), b0 = read_lane(bw, 0);
      // the walk over the windows: iteration x reads on the left iff A(i) <= B(j)
      uint32_t di = 0, dj = 0;
      for (uint32_t x = 0; x < ns; x++) {
        const uint64_t a = read_lane(aw, (int)di), bb = read_lane(bw, (int)dj);
        const bool left = a <= bb;
        if (lane == 0) sh_blk[x] = left ? (uint32_t)(i0 + di + 1) : (uint32_t)(nl - (j0 + dj));
        if (left) di++;
        else dj++;
      }
      // left keys stored before iteration s0: those of the first i0 and the last j0 blocks
      if (lane == 0) sh_lc0 = ns ? (uint64_t)IP_B * i0 - a0 + b0 : Q;
    }
    __syncthreads();
    const uint64_t lc0 = sh_lc0, rc0 = (uint64_t)IP_B * s0 - lc0;
    // 2. load the tile's vectors (all loads issued first), count their left keys
    R kv[VPW];
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const uint32_t qq = q < ns * IP_U ? q : 0u;
      const uint64_t pos = ms + (uint64_t)sh_blk[qq / IP_U] * IP_B + (qq % IP_U) * IP_V + lane;
      kv[r] = q < ns * IP_U ? ip_load<K>(keys, pos, tmode) : K::maxv();
    }
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const uint64_t lm = ballot(q < ns * IP_U && ip_left<K>(kv[r], pv, strict));
      if (lane == 0 && q < ns * IP_U) sh_vc[q] = (uint32_t)__popcll(lm);
    }
    __syncthreads();   // every wave has its keys: the tile has read its blocks
    if (w == 0) {
      // publish "loaded", then wait until every earlier tile of the range has too
      if (lane == 0 && t != 0) ip_publish(p, g, epoch | IP_ST_AGG);
      (void)ip_lookback(p, g, g0, epoch);
      if (lane == 0) ip_publish(p, g, epoch | IP_ST_INC);
    } else if (w == 1) {
      // staging offsets: left keys exclusive, right keys inclusive (vector order)
      uint32_t cl[VPL], cr[VPL], sl = 0, sr = 0;
#pragma unroll
      for (int u = 0; u < VPL; u++) {
        const uint32_t q = (uint32_t)lane * VPL + u;
        const uint32_t c = q < ns * IP_U ? sh_vc[q] : 0u;
        cl[u] = c;
        cr[u] = q < ns * IP_U ? IP_V - c : 0u;
        sl += cl[u];
        sr += cr[u];
      }
      const uint64_t il = wave_incl_scan64(sl), irr = wave_incl_scan64(sr);
      uint32_t bl = (uint32_t)(il - sl), br = (uint32_t)(irr - sr);
#pragma unroll
      for (int u = 0; u < VPL; u++) {
        const uint32_t q = (uint32_t)lane * VPL + u;
        br += cr[u];
        if (q < NV) {
          sh_vlo[q] = bl;
          sh_vro[q] = br;
        }
        bl += cl[u];
      }
      if (lane == WAVE - 1) sh_nlt = (uint32_t)il;
    }
    __syncthreads();
    const uint32_t nlt = sh_nlt, nvalid = ns * IP_B, nrt = nvalid - nlt;
    // 3. stage: left keys in iteration order from 0; right keys from the top down in
    // iteration order (a vector's right keys in lane order)
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const bool left = ip_left<K>(kv[r], pv, strict);
      const uint32_t lr = mbcnt(ballot(left));
      if (q < ns * IP_U) {
        const uint32_t d = left ? sh_vlo[q] + lr : nvalid - sh_vro[q] + ((uint32_t)lane - lr);
        stage[d] = ip_s<K>(kv[r]);
      }
    }
    __syncthreads();
    // 4. write the tile's two runs (internal form), the remainder (tile 0) and the
    // held-back blocks (last tile: every tile of the range has loaded)
    TW::write_run(stage, keys, 0, nlt, ms + lc0, 0, p.n_total, p.off);
    TW::write_run(stage, keys, nlt, nrt, me - rc0 - nrt, 0, p.n_total, p.off);
    const S* sv = (const S*)p.ip_stash + (uint64_t)si * IP_STASH;
    auto saved = [&](uint32_t i) -> R { return ip_load<K>(sv, i, 0); };
    auto held = [&](uint32_t i) -> R { return ip_load<K>(sv, IP_B + i, 0); };
    if (t == 0 && w == 2) ip_store_remainder<K>(saved, store_key, sg.b, me, nrem, pv, strict);
    const bool last = t == nt - 1;
    // the last tile ends the loop: the loop's left keys are those before it and its own
    const uint64_t Q = lc0 + nlt;
    if (last) ip_store_held<K>(held, store_key, ms, me, Q, (uint64_t)IP_B * nl - Q, ir.cfirst, pv, strict, w);
    if (tid == 0) {
      nread += nvalid;
      nwritten += nvalid + (t == 0 ? nrem : 0u) + (last ? 2u * IP_B : 0u);
    }
    tiles_done++;
    if (last) {
      // the range is partitioned: plan what follows (as level_kernel, keys stay in the
      // caller's array in internal form)
      const uint64_t bound = ms + Q + ir.cfirst + ir.clast;
      const bool fb = (sg.flags & SEG_FALLBACK) != 0;
      const uint32_t cf = fb ? SEG_FALLBACK : 0u;
      if (tid == 0) {
        if (!fb) {
          atomicAdd(&p.stats->partitions, 1ull);
          atomicAdd(&p.stats->keys_partitioned, (unsigned long long)len);
          atomicMax(&p.stats->max_depth, (unsigned long long)sg.depth);
        } else {
          atomicAdd(&p.stats->fallback_partitions, 1ull);
        }
      }
      // keys of [fb_, fe_) all equal the pivot and are final: written back in the
      // caller's form when that differs from the internal one
      auto retire_equal = [&](uint64_t fb_, uint64_t fe_) {
        if (p.mode == 0 || fe_ <= fb_) return;
        const uint64_t nch = (fe_ - fb_ + FILL_CHUNK - 1) / FILL_CHUNK;
        if (tid == 0) {
          sh_fill0 = atomicAdd(&p.solo_ctr->count, (unsigned long long)nch);
          atomicAdd(&p.stats->solo_items, (unsigned long long)nch);
        }
        __syncthreads();
        uint64_t lo, hi;
        to_words<K>(pv, lo, hi);
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
        retire_equal(bound, sg.e);
        if (tid == 0) route<K, 1>(p, make_seg<K>(sg.b, bound, sg.depth + 1, sg.limit, cf, pv), L + 1);
      } else if (bound == sg.e && !fb) {
        // degenerate: the range minimum decides (Alg. 1, ScanMinMax), from the count
        // launch's tile minima and the prologue's minimum of the other keys
        R m = K::from_u64x2(ir.mn_lo, ir.mn_hi);
        for (unsigned long long tt = g0 + tid; tt < g0 + nt; tt += LEVEL_P)
          m = K::kmin(m, K::from_u64x2(p.tilemin[tt].lo, p.tilemin[tt].hi));
        m = wave_min<K>(m);
        if (lane == 0) sh_wmin[w] = m;
        __syncthreads();
        if (tid == 0) {
          R mm = sh_wmin[0];
          for (int ww = 1; ww < NW; ww++) mm = K::kmin(mm, sh_wmin[ww]);
          sh_segmin = mm;
        }
        __syncthreads();
        const R mn = sh_segmin;
        if (tid == 0) atomicAdd(&p.stats->degenerate, 1ull);
        if (K::eq(mn, pv)) {
          if (tid == 0) atomicAdd(&p.stats->all_equal, 1ull);
          retire_equal(sg.b, sg.e);
        } else if (tid == 0) {
          route<K, 1>(p, make_seg<K>(sg.b, sg.e, sg.depth + 1, sg.limit, cf | SEG_OVERRIDE | SEG_PIVOT, mn), L + 1);
        }
      } else if (bound == sg.e) {
        if (tid == 0)
          route<K, 1>(p, make_seg<K>(sg.b, sg.e, sg.depth + 1, sg.limit, cf | SEG_OVERRIDE | SEG_PIVOT | SEG_STRICT, pv),
                      L + 1);
      } else if (tid == 0) {
        route<K, 1>(p, make_seg<K>(sg.b, bound, sg.depth + 1, sg.limit, cf, pv), L + 1);
        route<K, 1>(p, make_seg<K>(bound, sg.e, sg.depth + 1, sg.limit, cf, pv), L + 1);
      }
    }
    __syncthreads();
  }
  if (tid == 0 && tiles_done) {
    atomicAdd(&p.stats->level_tiles, tiles_done);
    atomicAdd(&p.stats->hbm_read_keys, nread);
    atomicAdd(&p.stats->hbm_write_keys, nwritten);
  }
}

// ---- in-place partitions of one workgroup (the solo kernel's global partitions) ----------

// Partition keys[b, e) (e - b <= IP_SOLO_MAX keys; tmode: transform on
// reading) in place by the workgroup, in the order above: a counting pass (the
// remainder, the held-back blocks into LDS, the left count of every loop block), every
// loop block's iteration from its merge rank, then the iterations in chunks of
// ip_steps blocks, each read into LDS before it is written (its stores land on keys
// read by it or earlier).  lds: the workgroup's two LDS key buffers (bufA stages a
// chunk; bufB holds the saved keys in its first half and the block tables in its
// second).  Returns the bound; *mn gets the range minimum.  Ends with a barrier.
template <class K, int P>
__device__ uint64_t ip_partition_workgroup(typename K::S* keys, uint64_t b, uint64_t e, typename K::R pv, bool strict,
                                           int tmode, typename K::S* bufA, typename K::S* bufB, typename K::R* mn) {
  using R = typename K::R;
  using S = typename K::S;
  constexpr uint32_t CS = ip_chunk_steps(K::SIZE);  // iterations per chunk
  constexpr uint32_t NV = CS * IP_U;
  constexpr int NW = P / WAVE;
  constexpr int VPW = (int)((NV + NW - 1) / NW);
  constexpr int VPL = (int)((NV + WAVE - 1) / WAVE);
  constexpr uint32_t MAXB = (uint32_t)(IP_SOLO_MAX / IP_B);
  static_assert(IP_STASH * sizeof(S) <= LOCAL_BYTES / 2, "saved keys fit half an LDS buffer");
  static_assert(CS * IP_B * sizeof(S) <= LOCAL_BYTES, "a chunk fits one LDS buffer");
  using TW = Tile<K, P, 1>;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
  // tables in bufB's second half
  uint32_t* cnt = (uint32_t*)((char*)bufB + LOCAL_BYTES / 2);   // MAXB + 2: loop blocks, [MAXB], [MAXB+1]: held back
  uint32_t* pfx = cnt + MAXB + 2;                               // MAXB + 1: pfx[k], k = 0..nl
  uint32_t* blk = pfx + MAXB + 1;                               // MAXB: block read at each iteration
  uint32_t* vc = blk + MAXB;                                    // NV per chunk: vector left counts
  uint32_t* vlo = vc + NV;
  uint32_t* vro = vlo + NV;
  uint32_t* misc = vro + NV;                                    // [0] lrem, [1] chunk left total
  R* wmin = (R*)(((uintptr_t)(misc + 4) + 15) & ~(uintptr_t)15);
  static_assert((MAXB + 2 + MAXB + 1 + MAXB + 3 * NV + 4) * 4 + 16 + NW * sizeof(R) <= LOCAL_BYTES / 2,
                "block tables fit");
  S* sv = bufB;   // [0, nrem) remainder, [IP_B, 3 IP_B) held-back blocks

  const uint64_t len = e - b;
  if (len < 2 * IP_B) {
    // the small loop alone: a stable split (wave 0 holds the keys in registers)
    constexpr int SR = 2 * IP_B / WAVE;
    if (w == 0) {
      R x[SR];
      R m0 = K::maxv();
#pragma unroll
      for (int u = 0; u < SR; u++) {
        const uint32_t i = (uint32_t)(u * WAVE + lane);
        x[u] = ip_load<K>(keys, b + (i < len ? i : 0u), tmode);
        if (i < len) m0 = K::kmin(m0, x[u]);
      }
      uint32_t c = 0;
#pragma unroll
      for (int u = 0; u < SR; u++)
        c += (uint32_t)__popcll(ballot((uint32_t)(u * WAVE + lane) < len && ip_left<K>(x[u], pv, strict)));
      uint32_t l = 0, r = 0;
#pragma unroll
      for (int u = 0; u < SR; u++) {
        const bool valid = (uint32_t)(u * WAVE + lane) < len;
        const bool left = valid && ip_left<K>(x[u], pv, strict);
        const uint64_t ml = ballot(left), mr = ballot(valid && !left);
        if (left) keys[b + l + mbcnt(ml)] = ip_s<K>(x[u]);
        else if (valid) keys[b + c + r + mbcnt(mr)] = ip_s<K>(x[u]);
        l += (uint32_t)__popcll(ml);
        r += (uint32_t)__popcll(mr);
      }
      m0 = wave_min<K>(m0);
      if (lane == 0) {
        misc[0] = c;
        wmin[0] = m0;
      }
    }
    __syncthreads();
    *mn = wmin[0];
    const uint64_t bound = b + misc[0];
    __syncthreads();
    return bound;
  }
  const uint32_t nrem = (uint32_t)(len % IP_B);
  const uint32_t nl = (uint32_t)ip_loop_blocks(len);
  R m = K::maxv();
  for (uint32_t k = (uint32_t)tid; k < nl + 2; k += P) cnt[k < nl ? k : MAXB + (k - nl)] = 0;
  if (w == 0) {
    uint32_t c = 0;
    for (uint32_t x0 = 0; x0 < nrem; x0 += WAVE) {
      const bool valid = x0 + (uint32_t)lane < nrem;
      const R x = ip_load<K>(keys, b + (valid ? x0 + (uint32_t)lane : 0u), tmode);
      if (valid) {
        sv[x0 + lane] = ip_s<K>(x);
        m = K::kmin(m, x);
      }
      c += (uint32_t)__popcll(ballot(valid && ip_left<K>(x, pv, strict)));
    }
    if (lane == 0) misc[0] = c;
  }
  __syncthreads();
  const uint32_t lrem = misc[0], rrem = nrem - lrem;
  const uint64_t ms = b + lrem, me = e - rrem;
  // counting pass: held-back blocks (saved) and loop blocks (vectors by waves)
  for (uint32_t q = (uint32_t)w; q < (nl + 2) * IP_U; q += NW) {
    const uint32_t kb = q / IP_U, v = q % IP_U;   // kb < nl: loop block kb + 1; then first, last
    uint64_t pos;
    if (kb < nl) {
      pos = ms + (uint64_t)(kb + 1) * IP_B + v * IP_V + lane;
    } else {
      const uint32_t y = v * IP_V + (uint32_t)lane;
      pos = kb == nl ? (y < rrem ? me + y : ms + y) : me - IP_B + y;
    }
    const R x = ip_load<K>(keys, pos, tmode);
    m = K::kmin(m, x);
    if (kb >= nl) sv[IP_B + (kb - nl) * IP_B + v * IP_V + lane] = ip_s<K>(x);
    const uint32_t c = (uint32_t)__popcll(ballot(ip_left<K>(x, pv, strict)));
    if (lane == 0) atomicAdd(&cnt[kb < nl ? kb : MAXB + (kb - nl)], c);
  }
  m = wave_min<K>(m);
  if (lane == 0) wmin[w] = m;
  __syncthreads();
  // prefix of the loop blocks' left counts (wave 0): pfx[k] = blocks 1..k
  if (w == 0) {
    constexpr int PL = (int)(MAXB / WAVE);
    uint32_t c[PL], s = 0;
#pragma unroll
    for (int u = 0; u < PL; u++) {
      const uint32_t k = (uint32_t)lane * PL + u;
      c[u] = k < nl ? cnt[k] : 0u;
      s += c[u];
    }
    uint32_t run = (uint32_t)wave_incl_scan64(s) - s;
#pragma unroll
    for (int u = 0; u < PL; u++) {
      const uint32_t k = (uint32_t)lane * PL + u;
      run += c[u];
      if (k < nl) pfx[k + 1] = run;
    }
    if (lane == 0) pfx[0] = 0;
  }
  __syncthreads();
  const uint32_t Q = pfx[nl];
  // merge rank of every loop block: k read on the left as block i = k - 1 at
  // i + #{j : B(j) < A(i)}, or on the right as block j = nl - k at j + #{i : A(i) <= B(j)}
  auto A = [&](uint32_t i) -> uint32_t { return (uint32_t)IP_B * i - pfx[i]; };
  auto Bq = [&](uint32_t j) -> uint32_t { return Q - pfx[nl - j]; };
  for (uint32_t k = (uint32_t)tid + 1; k <= nl; k += P) {
    const uint32_t ai = A(k - 1);
    uint32_t lo = 0, hi = nl;   // #{j < nl : B(j) < ai}
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      if (Bq(mid) < ai) lo = mid + 1;
      else hi = mid;
    }
    uint32_t step = (k - 1) + lo;
    if (step >= nl) {
      const uint32_t bj = Bq(nl - k);
      lo = 0;
      hi = nl;   // #{i < nl : A(i) <= bj}
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (A(mid) <= bj) lo = mid + 1;
        else hi = mid;
      }
      step = (nl - k) + lo;
    }
    blk[step] = k;
  }
  // the remainder's stores (their places were read above)
  if (w == 0) {
    auto saved = [&](uint32_t i) -> R { return (R)sv[i]; };
    auto st = [&](uint64_t i, R x) { keys[i] = ip_s<K>(x); };
    ip_store_remainder<K>(saved, st, b, me, nrem, pv, strict);
  }
  __syncthreads();
  // the iterations, a chunk at a time
  uint64_t lc = 0, rc = 0;
  for (uint32_t s0 = 0; s0 < nl; s0 += CS) {
    const uint32_t ns = nl - s0 < CS ? nl - s0 : CS;
    R kv[VPW];
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const uint32_t qq = q < ns * IP_U ? q : 0u;
      const uint64_t pos = ms + (uint64_t)blk[s0 + qq / IP_U] * IP_B + (qq % IP_U) * IP_V + lane;
      kv[r] = q < ns * IP_U ? ip_load<K>(keys, pos, tmode) : K::maxv();
    }
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const uint64_t lm = ballot(q < ns * IP_U && ip_left<K>(kv[r], pv, strict));
      if (lane == 0 && q < ns * IP_U) vc[q] = (uint32_t)__popcll(lm);
    }
    __syncthreads();
    if (w == 0) {
      uint32_t cl[VPL], cr[VPL], sl = 0, sr = 0;
#pragma unroll
      for (int u = 0; u < VPL; u++) {
        const uint32_t q = (uint32_t)lane * VPL + u;
        cl[u] = q < ns * IP_U ? vc[q] : 0u;
        cr[u] = q < ns * IP_U ? IP_V - cl[u] : 0u;
        sl += cl[u];
        sr += cr[u];
      }
      const uint64_t il = wave_incl_scan64(sl), irr = wave_incl_scan64(sr);
      uint32_t bl = (uint32_t)(il - sl), br = (uint32_t)(irr - sr);
#pragma unroll
      for (int u = 0; u < VPL; u++) {
        const uint32_t q = (uint32_t)lane * VPL + u;
        br += cr[u];
        if (q < NV) {
          vlo[q] = bl;
          vro[q] = br;
        }
        bl += cl[u];
      }
      if (lane == WAVE - 1) misc[1] = (uint32_t)il;
    }
    __syncthreads();
    const uint32_t nlt = misc[1], nvalid = ns * IP_B, nrt = nvalid - nlt;
#pragma unroll
    for (int r = 0; r < VPW; r++) {
      const uint32_t q = (uint32_t)w + (uint32_t)r * NW;
      const bool left = ip_left<K>(kv[r], pv, strict);
      const uint32_t lr = mbcnt(ballot(left));
      if (q < ns * IP_U) bufA[left ? vlo[q] + lr : nvalid - vro[q] + ((uint32_t)lane - lr)] = ip_s<K>(kv[r]);
    }
    __syncthreads();
    TW::write_out_keys(bufA, keys, nlt, nvalid, ms + lc, me - rc - nrt, 0, ~0ull);
    lc += nlt;
    rc += nrt;
    __syncthreads();
  }
  // the held-back blocks
  {
    auto held = [&](uint32_t i) -> R { return (R)sv[IP_B + i]; };
    auto st = [&](uint64_t i, R x) { keys[i] = ip_s<K>(x); };
    ip_store_held<K>(held, st, ms, me, lc, rc, cnt[MAXB], pv, strict, w);
  }
  R mm = wmin[0];
#pragma unroll
  for (int ww = 1; ww < NW; ww++) mm = K::kmin(mm, wmin[ww]);
  *mn = mm;
  const uint64_t bound = ms + Q + cnt[MAXB] + cnt[MAXB + 1];
  __syncthreads();
  return bound;
}

// ---- in-place order in LDS (one wave) ------------------------------------------------------

// Partition s[lb, le) (le - lb <= 64 blocks) into d[lb, le) by one wave in the in-place
// order (the destinations the sequential scan would give; s and d are separate LDS
// buffers).  Block k's counts live in lane k.  Returns the bound; mn gets the range
// minimum (wave-uniform).
template <class K>
__device__ uint32_t ip_partition_wave(const typename K::S* s, typename K::S* d, uint32_t lb, uint32_t le,
                                      typename K::R pv, bool strict, typename K::R& mn) {
  using R = typename K::R;
  const int lane = lane_id();
  const uint32_t n = le - lb;
  R m = K::maxv();
  auto ld = [&](uint32_t i) -> R { return (R)s[i]; };
  auto st = [&](uint32_t i, R x) { d[i] = ip_s<K>(x); };
  if (n < 2 * IP_B) {
    // the small loop alone: a stable split
    uint32_t nlt = 0;
    for (uint32_t x0 = 0; x0 < n; x0 += WAVE) {
      const bool valid = x0 + (uint32_t)lane < n;
      const R x = ld(lb + (valid ? x0 + (uint32_t)lane : 0u));
      if (valid) m = K::kmin(m, x);
      nlt += (uint32_t)__popcll(ballot(valid && ip_left<K>(x, pv, strict)));
    }
    uint32_t l = 0, r = 0;
    for (uint32_t x0 = 0; x0 < n; x0 += WAVE) {
      const bool valid = x0 + (uint32_t)lane < n;
      const R x = ld(lb + (valid ? x0 + (uint32_t)lane : 0u));
      const bool left = valid && ip_left<K>(x, pv, strict);
      const uint64_t ml = ballot(left), mr = ballot(valid && !left);
      if (left) st(lb + l + mbcnt(ml), x);
      else if (valid) st(lb + nlt + r + mbcnt(mr), x);
      l += (uint32_t)__popcll(ml);
      r += (uint32_t)__popcll(mr);
    }
    mn = wave_min<K>(m);
    return lb + nlt;
  }
  const uint32_t nrem = n % IP_B, mb = n / IP_B, nl = mb - 2;
  uint32_t lrem = 0;
  for (uint32_t x0 = 0; x0 < nrem; x0 += WAVE) {
    const bool valid = x0 + (uint32_t)lane < nrem;
    const R x = ld(lb + (valid ? x0 + (uint32_t)lane : 0u));
    if (valid) m = K::kmin(m, x);
    lrem += (uint32_t)__popcll(ballot(valid && ip_left<K>(x, pv, strict)));
  }
  const uint32_t rrem = nrem - lrem, ms = lb + lrem, me = le - rrem;
  // main index t: the range's last rrem keys first, then the keys after the remainder
  auto at = [&](uint32_t t) -> uint32_t { return t < rrem ? me + t : ms + t; };
  uint32_t c4[IP_U] = {0u, 0u, 0u, 0u};
  for (uint32_t k = 0; k < mb; k++) {
#pragma unroll
    for (int v = 0; v < IP_U; v++) {
      const R x = ld(at(k * IP_B + v * IP_V + (uint32_t)lane));
      m = K::kmin(m, x);
      const uint32_t c = (uint32_t)__popcll(ballot(ip_left<K>(x, pv, strict)));
      if ((uint32_t)lane == k) c4[v] = c;
    }
  }
  const uint32_t ck = c4[0] + c4[1] + c4[2] + c4[3];
  // P[k] = left keys of loop blocks 1..k, in lane k
  const uint32_t P = (uint32_t)wave_incl_scan64((lane >= 1 && (uint32_t)lane <= nl) ? ck : 0u);
  const uint32_t Q = read_lane(P, (int)nl);
  const uint32_t k = (uint32_t)lane;
  const uint32_t pkm1 = (uint32_t)__shfl((int)P, lane >= 1 ? lane - 1 : 0);
  const uint32_t ai = (uint32_t)IP_B * (k - 1) - pkm1;   // as left block i = k - 1
  const uint32_t bj = Q - P;                             // as right block j = nl - k
  uint32_t cb = 0, ca = 0;
  for (uint32_t x = 0; x < nl; x++) {
    const uint32_t Ax = (uint32_t)IP_B * x - read_lane(P, (int)x);
    const uint32_t Bx = Q - read_lane(P, (int)(nl - x));
    cb += Bx < ai ? 1u : 0u;
    ca += Ax <= bj ? 1u : 0u;
  }
  // lane k's block: its iteration and the left keys stored before it (loop blocks:
  // those of the i blocks read on the left and the j on the right before it; the
  // held-back blocks, first then last, come after the loop)
  const bool loop_blk = k >= 1 && k <= nl;
  const uint32_t pa = (k - 1) + cb;
  const bool from_left = pa < nl;
  const uint32_t step = loop_blk ? (from_left ? pa : (nl - k) + ca) : (k == 0 ? nl : nl + 1);
  const uint32_t i = loop_blk ? (from_left ? k - 1 : step - (nl - k)) : 0u;
  const uint32_t j = loop_blk ? step - i : 0u;
  const uint32_t pi = (uint32_t)__shfl((int)P, (int)(i & (WAVE - 1)));
  const uint32_t pj = (uint32_t)__shfl((int)P, (int)((nl - j) & (WAVE - 1)));
  const uint32_t ck0 = read_lane(ck, 0);
  const uint32_t lcb = loop_blk ? pi + (Q - pj) : Q + (k == 0 ? 0u : ck0);
  const uint32_t rcb = (uint32_t)IP_B * step - lcb;
  for (uint32_t kb = 0; kb < mb; kb++) {
    const uint32_t l0 = read_lane(lcb, (int)kb), r0 = read_lane(rcb, (int)kb);
    uint32_t l = 0, r = 0;
#pragma unroll
    for (int v = 0; v < IP_U; v++) {
      const R x = ld(at(kb * IP_B + v * IP_V + (uint32_t)lane));
      const uint32_t nlv = ip_store_vector<K>(x, ip_left<K>(x, pv, strict), st, ms + l0 + l, me - r0 - r);
      l += nlv;
      r += IP_V - nlv;
    }
  }
  auto rem = [&](uint32_t i) -> R { return ld(lb + i); };
  ip_store_remainder<K>(rem, st, lb, me, nrem, pv, strict);
  mn = wave_min<K>(m);
  return ms + Q + read_lane(ck, 0) + read_lane(ck, (int)(mb - 1));
}

// Partition s[lb, le) into d[lb, le) in the in-place order by a group of G waves (this
// wave is number sw of its group; go: the group has a range).  Every wave of the
// workgroup calls it: it holds two barriers.  The group's waves count the blocks
// k = sw, sw + G, ... (a vector's left count in tab[4k + v]); wave 0 of the group gives
// every block its merge rank and offsets (lane k, into the table's second half) and
// the bound; then the waves store their blocks, wave 0 also the remainder.  A range
// under two blocks is split by wave 0 alone.  tab: 512 bytes of LDS for the group.
// Returns the bound (wave 0 of the group); mn gets the wave's minimum of what it read.
template <class K>
__device__ uint32_t ip_partition_group(const typename K::S* s, typename K::S* d, uint32_t lb, uint32_t le,
                                       typename K::R pv, bool strict, int G, int sw, bool go, uint8_t* tab,
                                       typename K::R& mn) {
  using R = typename K::R;
  const int lane = lane_id();
  const uint32_t n = go ? le - lb : 0u;
  R m = K::maxv();
  auto ld = [&](uint32_t i) -> R { return (R)s[i]; };
  auto st = [&](uint32_t i, R x) { d[i] = ip_s<K>(x); };
  uint16_t* off = reinterpret_cast<uint16_t*>(tab + 256);   // block k: [2k] left, [2k + 1] right keys before it
  uint32_t bound = lb;
  const bool small = n < 2 * IP_B;
  const uint32_t nrem = n % IP_B, mb = n / IP_B, nl = mb >= 2 ? mb - 2 : 0u;
  uint32_t lrem = 0;
  if (go && !small) {
    for (uint32_t x0 = 0; x0 < nrem; x0 += WAVE) {
      const bool valid = x0 + (uint32_t)lane < nrem;
      const R x = ld(lb + (valid ? x0 + (uint32_t)lane : 0u));
      if (valid && sw == 0) m = K::kmin(m, x);
      lrem += (uint32_t)__popcll(ballot(valid && ip_left<K>(x, pv, strict)));
    }
  }
  const uint32_t rrem = nrem - lrem, ms = lb + lrem, me = le - rrem;
  auto at = [&](uint32_t t) -> uint32_t { return t < rrem ? me + t : ms + t; };
  // 1. counts
  if (go && !small) {
    for (uint32_t k = (uint32_t)sw; k < mb; k += (uint32_t)G) {
#pragma unroll
      for (int v = 0; v < IP_U; v++) {
        const R x = ld(at(k * IP_B + v * IP_V + (uint32_t)lane));
        m = K::kmin(m, x);
        const uint32_t c = (uint32_t)__popcll(ballot(ip_left<K>(x, pv, strict)));
        if (lane == 0) tab[4 * k + v] = (uint8_t)c;
      }
    }
  }
  __syncthreads();
  // 2. ranks and offsets (wave 0 of the group; lane k = block k); the small split
  if (go && sw == 0) {
    if (small) {
      bound = ip_partition_wave<K>(s, d, lb, le, pv, strict, m);
    } else {
      const uint32_t k = (uint32_t)lane;
      uint32_t c4[IP_U];
#pragma unroll
      for (int v = 0; v < IP_U; v++) c4[v] = k < mb ? tab[4 * k + v] : 0u;
      const uint32_t ck = c4[0] + c4[1] + c4[2] + c4[3];
      const uint32_t P = (uint32_t)wave_incl_scan64((lane >= 1 && k <= nl) ? ck : 0u);
      const uint32_t Q = read_lane(P, (int)nl);
      const uint32_t pkm1 = (uint32_t)__shfl((int)P, lane >= 1 ? lane - 1 : 0);
      const uint32_t ai = (uint32_t)IP_B * (k - 1) - pkm1;
      const uint32_t bj = Q - P;
      uint32_t cb = 0, ca = 0;
      for (uint32_t x = 0; x < nl; x++) {
        const uint32_t Ax = (uint32_t)IP_B * x - read_lane(P, (int)x);
        const uint32_t Bx = Q - read_lane(P, (int)(nl - x));
        cb += Bx < ai ? 1u : 0u;
        ca += Ax <= bj ? 1u : 0u;
      }
      const bool loop_blk = k >= 1 && k <= nl;
      const uint32_t pa = (k - 1) + cb;
      const bool from_left = pa < nl;
      const uint32_t step = loop_blk ? (from_left ? pa : (nl - k) + ca) : (k == 0 ? nl : nl + 1);
      const uint32_t i = loop_blk ? (from_left ? k - 1 : step - (nl - k)) : 0u;
      const uint32_t j = loop_blk ? step - i : 0u;
      const uint32_t pi = (uint32_t)__shfl((int)P, (int)(i & (WAVE - 1)));
      const uint32_t pj = (uint32_t)__shfl((int)P, (int)((nl - j) & (WAVE - 1)));
      const uint32_t ck0 = read_lane(ck, 0);
      const uint32_t lcb = loop_blk ? pi + (Q - pj) : Q + (k == 0 ? 0u : ck0);
      if (k < mb) {
        off[2 * k] = (uint16_t)lcb;
        off[2 * k + 1] = (uint16_t)((uint32_t)IP_B * step - lcb);
      }
      bound = ms + Q + ck0 + read_lane(ck, (int)(mb - 1));
    }
  }
  __syncthreads();
  // 3. stores
  if (go && !small) {
    for (uint32_t k = (uint32_t)sw; k < mb; k += (uint32_t)G) {
      const uint32_t l0 = off[2 * k], r0 = off[2 * k + 1];
      uint32_t l = 0, r = 0;
#pragma unroll
      for (int v = 0; v < IP_U; v++) {
        const R x = ld(at(k * IP_B + v * IP_V + (uint32_t)lane));
        const uint32_t nlv = ip_store_vector<K>(x, ip_left<K>(x, pv, strict), st, ms + l0 + l, me - r0 - r);
        l += nlv;
        r += IP_V - nlv;
      }
    }
    if (sw == 0) {
      auto rem = [&](uint32_t i2) -> R { return ld(lb + i2); };
      ip_store_remainder<K>(rem, st, lb, me, nrem, pv, strict);
    }
  }
  mn = wave_min<K>(m);
  return bound;
}

// ---- bounded-time sort in place ---------------------------------------------------------

// Half-cleaner stages d = top .. 2 (pairs i, i + d/2 inside aligned blocks of d) of
// a[0, n) in LDS by the workgroup; positions >= n act as +inf.
template <class K, class S>
__device__ void wg_halfclean_lds(S* a, uint32_t n, uint32_t top) {
  using R = typename K::R;
  for (uint32_t dd = top; dd >= 2; dd >>= 1) {
    const uint32_t half = dd >> 1;
    for (uint32_t idx = threadIdx.x; idx < (top / 2) * ((n + top - 1) / top); idx += blockDim.x) {
      const uint32_t i = (idx / half) * dd + (idx % half), j = i + half;
      if (j < n) {
        const R x = (R)a[i], y = (R)a[j];
        if (K::lt(y, x)) {
          a[i] = (S)y;
          a[j] = (S)x;
        }
      }
    }
    __syncthreads();
  }
}

// Bounded-time sort of keys[it.b, it.e) without key scratch: the flip-form bitonic
// sort, its stages run in LDS while their pairs lie in one chunk of C keys (C the
// largest power of two within the LDS capacity) and through global memory otherwise.
// O(n log^2 n) work.  The caller's array ends in the caller's form.  Thread 0 adds the
// keys its passes read and write to rd and wr.
template <class K>
__device__ void fallback_global_inplace(const Params& p, typename K::S* bufA, const Seg& it, unsigned long long& rd,
                                        unsigned long long& wr) {
  using R = typename K::R;
  using S = typename K::S;
  const uint64_t b = it.b, n = it.e - it.b;
  S* X = (S*)p.keys + b;
  const int tmode = (it.flags & SEG_RAW) ? p.mode : 0;
  if (threadIdx.x == 0) atomicAdd(&p.stats->bounded_global, 1ull);
  uint32_t C = 1;
  while ((uint64_t)C * 2 <= p.local_cap) C *= 2;
  uint64_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  auto pass = [&](uint64_t keys_moved) {
    if (threadIdx.x == 0) {
      rd += keys_moved;
      wr += keys_moved;
    }
  };
  // 1. chunks sorted in LDS (stages up to C), internal form
  for (uint64_t c0 = 0; c0 < n; c0 += C) {
    const uint32_t m = (uint32_t)(c0 + C < n ? C : n - c0);
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) bufA[i] = ip_s<K>(ip_load<K>(X, c0 + i, tmode));
    __syncthreads();
    wg_bitonic_lds<K, S>(bufA, m);
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) X[c0 + i] = bufA[i];
    __syncthreads();
  }
  pass(n);
  // 2. merges of 2C .. p2 keys: the stages over more than C keys in global memory,
  // then the rest of each merge chunk by chunk in LDS
  for (uint64_t kk = 2 * (uint64_t)C; kk <= p2; kk <<= 1) {
    for (uint64_t dd = kk; dd > C; dd >>= 1) {
      const uint64_t half = dd >> 1;
      for (uint64_t idx = threadIdx.x; idx < p2 / 2; idx += blockDim.x) {
        const uint64_t i = (idx / half) * dd + (idx % half);
        const uint64_t j = (dd == kk) ? (i ^ (dd - 1)) : (i + half);
        if (j < n) {
          const R x = (R)X[i], y = (R)X[j];
          if (K::lt(y, x)) {
            X[i] = (S)y;
            X[j] = (S)x;
          }
        }
      }
      __syncthreads();
      pass(n);
    }
    for (uint64_t c0 = 0; c0 < n; c0 += C) {
      const uint32_t m = (uint32_t)(c0 + C < n ? C : n - c0);
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) bufA[i] = X[c0 + i];
      __syncthreads();
      wg_halfclean_lds<K, S>(bufA, m, C);
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) X[c0 + i] = bufA[i];
      __syncthreads();
    }
    pass(n);
  }
  // 3. the caller's form
  if (p.mode != 0) {
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) X[i] = K::store_t((R)X[i], p.mode);
    __syncthreads();
    pass(n);
  }
}
