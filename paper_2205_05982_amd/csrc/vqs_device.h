// vqs_device.h -- device-side building blocks for gfx950 (CDNA4, wave64).
//
// Key traits: every key type is sorted internally as an unsigned integer in
// ascending order.  Floats are mapped to unsigned integers by the order-preserving
// bit transform (flip all bits of negatives, set the sign bit of non-negatives),
// signed integers by flipping the sign bit, and descending order is the bitwise
// complement, so one comparison serves every key type and both orders of Sec. 2.4.  The transform is applied when keys are first
// read from the caller's array and inverted when results are written back.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vqs_types.h"

namespace vqs {

constexpr int WAVE = 64;

template <int BITS>
struct Key;

template <>
struct Key<16> {
  using S = uint16_t;  // storage in memory / LDS
  using R = uint32_t;  // register form (zero-extended)
  static constexpr int SIZE = 2;
  static constexpr int V = 8;  // keys per 16-byte chunk
  __device__ static R load_t(S s, int mode) {
    R r = s;
    if (mode & MODE_SIGNED) r ^= 0x8000u;
    if (mode & MODE_DESC) r = (~r) & 0xFFFFu;
    return r;
  }
  __device__ static S store_t(R r, int mode) {
    if (mode & MODE_DESC) r = (~r) & 0xFFFFu;
    if (mode & MODE_SIGNED) r ^= 0x8000u;
    return (S)r;
  }
  __device__ static bool lt(R a, R b) { return a < b; }
  __device__ static bool eq(R a, R b) { return a == b; }
  __device__ static R maxv() { return 0xFFFFu; }
  __device__ static R kmin(R a, R b) { return a < b ? a : b; }
  __device__ static R kmax(R a, R b) { return a < b ? b : a; }
  __device__ static R sel(bool c, R a, R b) { return c ? a : b; }
  __device__ static R shfl(R v, int lane) { return (R)__shfl((int)v, lane); }
  __device__ static R shfl_xor(R v, int m) { return (R)__shfl_xor((int)v, m); }
  __device__ static void unpack(const uint4& c, R (&k)[V]) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
      k[2 * i] = w[i] & 0xFFFFu;
      k[2 * i + 1] = w[i] >> 16;
    }
  }
  __device__ static void to_u64x2(R r, uint64_t& lo, uint64_t& hi) { lo = r; hi = 0; }
  __device__ static R from_u64x2(uint64_t lo, uint64_t) { return (R)lo; }
};

template <>
struct Key<32> {
  using S = uint32_t;
  using R = uint32_t;
  static constexpr int SIZE = 4;
  static constexpr int V = 4;
  __device__ static R load_t(S s, int mode) {
    R r = s;
    if (mode & MODE_FLOAT) r = (r & 0x80000000u) ? ~r : (r | 0x80000000u);
    if (mode & MODE_SIGNED) r ^= 0x80000000u;
    if (mode & MODE_DESC) r = ~r;
    return r;
  }
  __device__ static S store_t(R r, int mode) {
    if (mode & MODE_DESC) r = ~r;
    if (mode & MODE_SIGNED) r ^= 0x80000000u;
    if (mode & MODE_FLOAT) r = (r & 0x80000000u) ? (r & 0x7FFFFFFFu) : ~r;
    return r;
  }
  __device__ static bool lt(R a, R b) { return a < b; }
  __device__ static bool eq(R a, R b) { return a == b; }
  __device__ static R maxv() { return 0xFFFFFFFFu; }
  __device__ static R kmin(R a, R b) { return a < b ? a : b; }
  __device__ static R kmax(R a, R b) { return a < b ? b : a; }
  __device__ static R sel(bool c, R a, R b) { return c ? a : b; }
  __device__ static R shfl(R v, int lane) { return (R)__shfl((int)v, lane); }
  __device__ static R shfl_xor(R v, int m) { return (R)__shfl_xor((int)v, m); }
  __device__ static void unpack(const uint4& c, R (&k)[V]) {
    k[0] = c.x;
    k[1] = c.y;
    k[2] = c.z;
    k[3] = c.w;
  }
  __device__ static void to_u64x2(R r, uint64_t& lo, uint64_t& hi) { lo = r; hi = 0; }
  __device__ static R from_u64x2(uint64_t lo, uint64_t) { return (R)lo; }
};

template <>
struct Key<64> {
  using S = uint64_t;
  using R = uint64_t;
  static constexpr int SIZE = 8;
  static constexpr int V = 2;
  __device__ static R load_t(S s, int mode) {
    R r = s;
    if (mode & MODE_FLOAT) r = (r >> 63) ? ~r : (r | 0x8000000000000000ull);
    if (mode & MODE_SIGNED) r ^= 0x8000000000000000ull;
    if (mode & MODE_DESC) r = ~r;
    return r;
  }
  __device__ static S store_t(R r, int mode) {
    if (mode & MODE_DESC) r = ~r;
    if (mode & MODE_SIGNED) r ^= 0x8000000000000000ull;
    if (mode & MODE_FLOAT) r = (r >> 63) ? (r & 0x7FFFFFFFFFFFFFFFull) : ~r;
    return r;
  }
  __device__ static bool lt(R a, R b) { return a < b; }
  __device__ static bool eq(R a, R b) { return a == b; }
  __device__ static R maxv() { return ~0ull; }
  __device__ static R kmin(R a, R b) { return a < b ? a : b; }
  __device__ static R kmax(R a, R b) { return a < b ? b : a; }
  __device__ static R sel(bool c, R a, R b) { return c ? a : b; }
  __device__ static R shfl(R v, int lane) {
    return ((R)(uint32_t)__shfl((int)(uint32_t)(v >> 32), lane) << 32) |
           (uint32_t)__shfl((int)(uint32_t)v, lane);
  }
  __device__ static R shfl_xor(R v, int m) {
    return ((R)(uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m) << 32) |
           (uint32_t)__shfl_xor((int)(uint32_t)v, m);
  }
  __device__ static void unpack(const uint4& c, R (&k)[V]) {
    k[0] = ((uint64_t)c.y << 32) | c.x;
    k[1] = ((uint64_t)c.w << 32) | c.z;
  }
  __device__ static void to_u64x2(R r, uint64_t& lo, uint64_t& hi) { lo = r; hi = 0; }
  __device__ static R from_u64x2(uint64_t lo, uint64_t) { return lo; }
};

// A key width together with the level kernels' tile size: LI 16-byte chunks per thread.
template <int BITS, int LI_>
struct KeyL;

// 128-bit keys: two 64-bit words, low word first in memory; compared as (hi, lo)
// lexicographically (Sec. 2.4, Alg. 2).
template <>
struct Key<128> {
  using S = u128k;
  using R = u128k;
  static constexpr int SIZE = 16;
  static constexpr int V = 1;
  __device__ static R load_t(S s, int mode) {
    if (mode & MODE_DESC) {
      s.lo = ~s.lo;
      s.hi = ~s.hi;
    }
    return s;
  }
  __device__ static S store_t(R r, int mode) { return load_t(r, mode); }
  __device__ static bool lt(R a, R b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
  __device__ static bool eq(R a, R b) { return a.hi == b.hi && a.lo == b.lo; }
  __device__ static R maxv() { return R{~0ull, ~0ull}; }
  // field-wise select: a select of whole structs becomes a select of their addresses,
  // which keeps them out of registers
  __device__ static R sel(bool c, R a, R b) { return R{c ? a.lo : b.lo, c ? a.hi : b.hi}; }
  __device__ static R kmin(R a, R b) { return sel(lt(b, a), b, a); }
  __device__ static R kmax(R a, R b) { return sel(lt(b, a), a, b); }
  __device__ static R shfl(R v, int lane) { return R{Key<64>::shfl(v.lo, lane), Key<64>::shfl(v.hi, lane)}; }
  __device__ static R shfl_xor(R v, int m) {
    return R{Key<64>::shfl_xor(v.lo, m), Key<64>::shfl_xor(v.hi, m)};
  }
  __device__ static void unpack(const uint4& c, R (&k)[V]) {
    k[0].lo = ((uint64_t)c.y << 32) | c.x;
    k[0].hi = ((uint64_t)c.w << 32) | c.z;
  }
  __device__ static void to_u64x2(R r, uint64_t& lo, uint64_t& hi) {
    lo = r.lo;
    hi = r.hi;
  }
  __device__ static R from_u64x2(uint64_t lo, uint64_t hi) { return R{lo, hi}; }
};

template <int BITS, int LI_>
struct KeyL : Key<BITS> {
  static constexpr int LI = LI_;
};

// ---- wave utilities ---------------------------------------------------------------

__device__ inline int lane_id() { return __lane_id(); }

// number of set bits of mask below this lane
__device__ inline uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// Lane exchange inside 16-lane rows, partner lane = lane ^ M, by DPP (data-parallel
// primitives: a VALU move with a lane pattern) where one exists: quad_perm for
// M = 1, 2, 3, row_half_mirror for M = 7, row_mirror for M = 15; ds_swizzle in
// bit mode for M = 4.
template <int M>
__device__ inline uint32_t xor_lanes32(uint32_t v) {
  static_assert(M == 1 || M == 2 || M == 3 || M == 4 || M == 7 || M == 15, "pattern");
  if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x1B, 0xF, 0xF, true);
  if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);
  if constexpr (M == 15) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true);
  // xor 4 = xor 7 (row_half_mirror) then xor 3 (quad_perm): two DPP moves, no LDS trip
  if constexpr (M == 4) return xor_lanes32<3>(xor_lanes32<7>(v));
  return v;
}

template <int M>
__device__ inline uint32_t xor_lanes(uint32_t v) { return xor_lanes32<M>(v); }

// The value of lane l (a constant lane), wave-uniform.
__device__ inline uint32_t read_lane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ inline uint64_t read_lane(uint64_t v, int l) {
  return ((uint64_t)read_lane((uint32_t)(v >> 32), l) << 32) | read_lane((uint32_t)v, l);
}
template <int M>
__device__ inline uint64_t xor_lanes(uint64_t v) {
  return ((uint64_t)xor_lanes32<M>((uint32_t)(v >> 32)) << 32) | xor_lanes32<M>((uint32_t)v);
}
template <int M>
__device__ inline u128k xor_lanes(u128k v) {
  return u128k{xor_lanes<M>(v.lo), xor_lanes<M>(v.hi)};
}
__device__ inline u128k read_lane(u128k v, int l) { return u128k{read_lane(v.lo, l), read_lane(v.hi, l)}; }

// ---- random numbers for the pivot sampler (Sec. 2.2) ---------------------------------

// SplitMix64 (Steele, Lea, Flood): golden-ratio increment, variant-13 finalizer.
__device__ inline uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// SFC64 (Doty-Humphrey), state a, b, c, counter.
struct Sfc64 {
  uint64_t a, b, c, w;
  __device__ uint64_t next() {
    const uint64_t out = a + b + w;
    w += 1;
    a = b ^ (b >> 11);
    b = c + (c << 3);
    c = ((c << 24) | (c >> 40)) + out;
    return out;
  }
};

// Sampler state of the range [b, e): SplitMix64 from the seed with b, then e, mixed
// in before the draws giving a, b, c; counter 1; twelve outputs discarded.
__device__ inline Sfc64 range_rng(uint64_t seed, uint64_t b, uint64_t e) {
  uint64_t x = seed;
  Sfc64 s;
  x ^= b;
  s.a = splitmix64(x);
  x ^= e;
  s.b = splitmix64(x);
  s.c = splitmix64(x);
  s.w = 1;
  for (int i = 0; i < 12; i++) (void)s.next();
  return s;
}

template <class K>
__device__ inline typename K::R med3(typename K::R x0, typename K::R x1, typename K::R x2) {
  // network (0,2) (0,1) (1,2): element 1 ends as the median
  typename K::R lo = K::kmin(x0, x2), hi = K::kmax(x0, x2);
  typename K::R m = K::kmax(lo, x1);
  return K::kmin(m, hi);
}

// ChoosePivot by one wave.  `load(i)` returns the key at position i relative to the
// range start (internal form).  b, e are the absolute range bounds (they seed the
// sampler).  Nine 64-byte chunks at random chunk offsets, lanewise medians of three of
// chunk groups, then reduction by medians of three (whole groups of W lanes while 3W
// remain, then consecutive triples, 0..2 leftovers dropped) until fewer than three
// remain; the first is the pivot.  All lanes return the pivot.
// A wave-uniform 64-bit value placed in scalar registers (lets the compiler run the
// sampler's integer arithmetic on the scalar unit).
__device__ inline uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// ChaCha20 block function (RFC 8439 Sec. 2.3): constants, 256-bit key, block counter,
// 96-bit nonce; 10 double rounds (columns, then diagonals) of the quarter round, then
// the input state added.  Only the first ten output words are produced.
__device__ inline uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

#define VQS_QR(a, b, c, d)     \
  a += b;                      \
  d = rotl32(d ^ a, 16);       \
  c += d;                      \
  b = rotl32(b ^ c, 12);       \
  a += b;                      \
  d = rotl32(d ^ a, 8);        \
  c += d;                      \
  b = rotl32(b ^ c, 7);

__device__ inline void chacha20_ten(const uint32_t (&key)[8], uint32_t counter, uint32_t n0, uint32_t n1,
                                    uint32_t n2, uint32_t (&u)[10]) {
  const uint32_t x[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, key[0], key[1], key[2], key[3],
                          key[4],      key[5],      key[6],      key[7],      counter, n0,     n1,     n2};
  uint32_t w0 = x[0], w1 = x[1], w2 = x[2], w3 = x[3], w4 = x[4], w5 = x[5], w6 = x[6], w7 = x[7];
  uint32_t w8 = x[8], w9 = x[9], w10 = x[10], w11 = x[11], w12 = x[12], w13 = x[13], w14 = x[14], w15 = x[15];
  for (int r = 0; r < 10; r++) {
    VQS_QR(w0, w4, w8, w12)
    VQS_QR(w1, w5, w9, w13)
    VQS_QR(w2, w6, w10, w14)
    VQS_QR(w3, w7, w11, w15)
    VQS_QR(w0, w5, w10, w15)
    VQS_QR(w1, w6, w11, w12)
    VQS_QR(w2, w7, w8, w13)
    VQS_QR(w3, w4, w9, w14)
  }
  u[0] = w0 + x[0];
  u[1] = w1 + x[1];
  u[2] = w2 + x[2];
  u[3] = w3 + x[3];
  u[4] = w4 + x[4];
  u[5] = w5 + x[5];
  u[6] = w6 + x[6];
  u[7] = w7 + x[7];
  u[8] = w8 + x[8];
  u[9] = w9 + x[9];
}
#undef VQS_QR

// The nine chunk starts (keys from the range start) ChoosePivot samples for [b, e):
// computed by each thread for its own range, so one wave can do it for 64 ranges.
// The ten 32-bit random values come from the range's SFC64 generator (five 64-bit
// draws, low half first), or, with the secure option, from the first ten words of the
// ChaCha20 block keyed by the caller's key with block counter = the low 32 bits of b
// and nonce = (the high 32 bits of b, the low and the high 32 bits of e).
template <class K>
__device__ inline void pivot_chunk_starts(uint64_t b, uint64_t e, const Params& p, uint64_t (&o)[9]) {
  constexpr int W = 64 / K::SIZE;
  const uint64_t nch = (e - b) / W;
  uint32_t u[10];
  if (p.rng_mode == 1) {
    chacha20_ten(p.rng_key, (uint32_t)b, (uint32_t)(b >> 32), (uint32_t)e, (uint32_t)(e >> 32), u);
  } else {
    Sfc64 rng = range_rng(p.seed, b, e);
#pragma unroll
    for (int i = 0; i < 5; i++) {
      const uint64_t r = rng.next();
      u[2 * i] = (uint32_t)r;
      u[2 * i + 1] = (uint32_t)(r >> 32);
    }
  }
#pragma unroll
  for (int i = 0; i < 9; i++) o[i] = (((uint64_t)u[i] * nch) >> 32) * W;
}

template <class K, class Load>
__device__ typename K::R choose_pivot_from(Load load, uint64_t o0, uint64_t o1, uint64_t o2, uint64_t o3,
                                           uint64_t o4, uint64_t o5, uint64_t o6, uint64_t o7, uint64_t o8);

template <class K, class Load>
__device__ typename K::R choose_pivot_wave(Load load, uint64_t b, uint64_t e, const Params& p) {
  b = uniform64(b);
  e = uniform64(e);
  uint64_t o[9];
  pivot_chunk_starts<K>(b, e, p, o);
  return choose_pivot_from<K>(load, o[0], o[1], o[2], o[3], o[4], o[5], o[6], o[7], o[8]);
}

// Lanewise medians of the nine sampled chunks, then the median reduction; the chunk
// starts are wave-uniform.
template <class K, class Load>
__device__ typename K::R choose_pivot_from(Load load, uint64_t o0, uint64_t o1, uint64_t o2, uint64_t o3,
                                           uint64_t o4, uint64_t o5, uint64_t o6, uint64_t o7, uint64_t o8) {
  using R = typename K::R;
  constexpr int W = 64 / K::SIZE;
  constexpr int M0 = 3 * W;               // 96, 48, 24 or 12 medians
  constexpr int NR = (M0 + WAVE - 1) / WAVE;
  const int lane = lane_id();

  // slot m lives in lane m % 64, register m / 64
  R v[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int m = r * WAVE + lane;
    v[r] = K::maxv();
    if (m < M0) {
      const int g = m / W, j = m % W;   // chunk group g uses chunks 3g, 3g+1, 3g+2
      const uint64_t c0 = g == 0 ? o0 : (g == 1 ? o3 : o6);
      const uint64_t c1 = g == 0 ? o1 : (g == 1 ? o4 : o7);
      const uint64_t c2 = g == 0 ? o2 : (g == 1 ? o5 : o8);
      R x0 = load(c0 + j), x1 = load(c1 + j), x2 = load(c2 + j);
      v[r] = med3<K>(x0, x1, x2);
    }
  }
  int cnt = M0;
  while (cnt >= 3) {
    const int nv = cnt / (3 * W);               // whole vector groups
    const int ns = (cnt - nv * 3 * W) / 3;      // then single triples
    const int outc = nv * W + ns;
    R nvv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
      const int o = r * WAVE + lane;
      int i0, d;
      if (o < nv * W) {
        i0 = (o / W) * 3 * W + (o % W);
        d = W;
      } else {
        i0 = nv * 3 * W + 3 * (o - nv * W);
        d = 1;
      }
      R x[3];
#pragma unroll
      for (int t = 0; t < 3; t++) {
        int idx = i0 + t * d;
        if (idx >= cnt) idx = 0;   // lanes beyond the outputs: any in-range slot
        R got = K::shfl(v[0], idx & (WAVE - 1));
#pragma unroll
        for (int rr = 1; rr < NR; rr++) {
          R g2 = K::shfl(v[rr], idx & (WAVE - 1));
          if ((idx >> 6) == rr) got = g2;
        }
        x[t] = got;
      }
      nvv[r] = med3<K>(x[0], x[1], x[2]);
    }
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = nvv[r];
    cnt = outc;
  }
  return K::shfl(v[0], 0);
}

}  // namespace vqs
