// vqs_learned.hip -- kernels of the learned 256-bucket splitter (u64 keys).
//
// Pipeline (host side in vqs_host.cpp): sample 1% of the keys in random aligned
// 64-byte chunks (the pivot sampler's unit); sort the sample with the plain method;
// mid-rank CDF targets; train the model with Adam in one workgroup; compile the
// monotone bucket map into 255 exact thresholds; 256-bin histograms per 65,536-key
// chunk; a per-bucket scan over the chunks; one scatter pass into 256 contiguous
// buckets; then the buckets are sorted as segments by the plain method.
//
// Every FP32 operation of the model's forward pass is a single correctly rounded
// operation in a fixed order (explicit fused multiply-adds, no contraction), so
// bucket ids are bit-identical to a scalar FP32 reference of the same steps.
#pragma clang fp contract(off)
#include "vqs_learned.h"
#include "vqs_device.h"

namespace vqs {

namespace {

// ---- model ------------------------------------------------------------------------

__device__ inline float clamp01(float a) { return fminf(fmaxf(a, 0.0f), 1.0f); }

// x(k): k rounded to float, its bit pattern as an unsigned integer, to float, * 2^-31
__device__ inline float key_to_x(uint64_t k) {
  const float f = __ull2float_rn(k);
  const uint32_t bits = __float_as_uint(f);
  return __fmul_rn(__uint2float_rn(bits), 0x1p-31f);
}

__device__ inline float mlp_forward(const float* P, float x) {
  const float xn = __fmul_rn(__fsub_rn(x, P[MLP_X0]), P[MLP_XS]);
  float h1[MLP_H];
#pragma unroll
  for (int i = 0; i < MLP_H; i++) h1[i] = clamp01(__fmaf_rn(P[MLP_W1 + i], xn, P[MLP_B1 + i]));
  float y = P[MLP_B3];
  for (int j = 0; j < MLP_H; j++) {
    float a = P[MLP_B2 + j];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) a = __fmaf_rn(P[MLP_W2 + j * MLP_H + i], h1[i], a);
    y = __fmaf_rn(P[MLP_W3 + j], clamp01(a), y);
  }
  return clamp01(y);
}

__device__ inline int bucket_of_y(float y) {
  const int b = (int)__fmul_rn(y, (float)NBUCKET);   // y in [0, 1]: exact scaling, then floor
  return b < NBUCKET - 1 ? b : NBUCKET - 1;
}

__device__ inline int mlp_bucket(const float* P, uint64_t k) { return bucket_of_y(mlp_forward(P, key_to_x(k))); }

// counter-based SplitMix64: output number c of the sequence started at seed
__device__ inline uint64_t splitmix_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The 255 thresholds of a classification sit in LDS in breadth-first order of the implicit
// binary search tree: level L (0..7) holds slots 2^L - 1 .. 2^(L+1) - 2, slot 2^L - 1 + j
// holding threshold (2j + 1) * 2^(7-L) - 1.  The nodes one search step can reach are then
// adjacent words, not words 2^(8-L) apart that all fall into the same LDS bank.
__device__ inline int tree_source(int slot) {
  const int L = 31 - __clz(slot + 1);
  const int j = slot + 1 - (1 << L);
  return (2 * j + 1) * (128 >> L) - 1;
}

__device__ inline void tree_load(uint64_t* E, const uint64_t* thr) {
  for (int i = threadIdx.x; i < NBUCKET - 1; i += blockDim.x) E[i] = thr[tree_source(i)];
}

// number of the first nvalid thresholds that are <= k (thresholds non-decreasing), by
// binary search over the tree: at level L the search stands at b, a multiple of 2^(8-L),
// and compares threshold b + 2^(7-L) - 1, the tree's node b >> (8-L) of that level.  Every
// level loads its node and selects without a branch, so that the searches of several keys
// of a thread interleave.
__device__ inline int classify(const uint64_t* E, int nvalid, uint64_t k) {
  int b = 0;
#pragma unroll
  for (int L = 0; L < 8; L++) {
    const int c = b + (128 >> L);
    const uint64_t e = E[(1 << L) - 1 + (b >> (8 - L))];
    b = ((c <= nvalid) & (e <= k)) ? c : b;
  }
  return b;
}

// ---- sampling and targets ----------------------------------------------------------

// chunk c: 8 keys (64 bytes) at chunk offset (u * chunks) >> 32, u the high half of
// SplitMix64 output c of the seed; chunks are counted from the array start
// (one thread per sampled key: eight neighbouring threads read and write a chunk's 64
// contiguous bytes)
__global__ void sample_kernel(const uint64_t* keys, uint64_t n, uint64_t* sample, uint64_t nsample_chunks,
                              uint64_t seed) {
  const uint64_t nch = n / 8;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsample_chunks * 8;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = i / 8;
    const uint32_t u = (uint32_t)(splitmix_at(seed, c) >> 32);
    const uint64_t off = (((uint64_t)u * nch) >> 32) * 8;
    sample[i] = keys[off + (i & 7)];
  }
}

// x(k) of each sorted sample and its mid-rank CDF target (first + last + 1) / 2 / m.
// The run of keys equal to s[i] is found by galloping outward from i (one load each
// way for a key without copies), then a binary search inside the last step.
__global__ void targets_kernel(const uint64_t* s, uint64_t m, float* x, float* t) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = s[i];
    // first: s[f] == k, then steps 1, 2, 4, ... down while the key is still k
    uint64_t f = i, step = 1;
    while (f >= step && s[f - step] == k) {
      f -= step;
      step <<= 1;
    }
    uint64_t lo = f >= step ? f - step + 1 : 0, hi = f;   // first index with s == k is in [lo, hi]
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (s[mid] < k) lo = mid + 1; else hi = mid;
    }
    const uint64_t first = lo;
    // last: the same upward
    uint64_t e = i;
    step = 1;
    while (e + step < m && s[e + step] == k) {
      e += step;
      step <<= 1;
    }
    lo = e;
    hi = e + step < m ? e + step - 1 : m - 1;   // last index with s == k is in [lo, hi]
    while (lo < hi) {
      const uint64_t mid = (lo + hi + 1) / 2;
      if (s[mid] == k) lo = mid; else hi = mid - 1;
    }
    const uint64_t last = lo;
    x[i] = key_to_x(k);
    t[i] = (float)(((double)first + (double)last + 1.0) * 0.5 / (double)m);
  }
}

// untrained model: unit ramps tiling xn in [0,1] (w1 = 32, b1 = -i), second layer
// (1 + 0.5 (u - 0.5)) / 32 with u from SplitMix64 outputs of the seed, biases
// 0.1 (u - 0.5), output weights 1/32; x0 = x of the smallest sample, xs = 1 / range
__global__ void init_kernel(float* P, uint64_t seed, const float* x, uint64_t m) {
  for (int i = threadIdx.x; i < MLP_NBLOCK; i += blockDim.x) {
    double v;
    if (i < MLP_B1) v = 32.0;
    else if (i < MLP_W2) v = -(double)(i - MLP_B1);
    else if (i < MLP_B2) {
      const double u = (double)(splitmix_at(seed, (uint64_t)(i - MLP_W2)) >> 40) / 16777216.0;
      v = (1.0 + 0.5 * (u - 0.5)) / 32.0;
    } else if (i < MLP_W3) {
      const double u = (double)(splitmix_at(seed, (uint64_t)(i - MLP_W2)) >> 40) / 16777216.0;
      v = 0.1 * (u - 0.5);
    } else if (i < MLP_B3) v = 1.0 / 32.0;
    else if (i == MLP_B3) v = 0.0;
    else if (i == MLP_X0) v = (double)x[0];
    else {
      const float r = __fsub_rn(x[m - 1], x[0]);
      v = (double)(r > 0.0f ? __fdiv_rn(1.0f, r) : 1.0f);
    }
    P[i] = (float)v;
  }
}

// ---- training ------------------------------------------------------------------------

// One workgroup of 512 threads trains on minibatches of up to 256 samples.  Thread t
// takes sample t % 256 and half t / 256 of the hidden units (both halves compute the
// first layer; each computes 16 second-layer units and 16 first-layer gradients).
// The weight-matrix gradient dL/dW2 = DA2^T H1 is a 32 x 256 x 32 product done in 4x4
// register tiles, one wave per group of 32 samples, then reduced over the groups.
constexpr int TRAIN_P = 512;
constexpr int TRAIN_NW = TRAIN_P / WAVE;       // 8 waves = 8 sample groups of 32
constexpr int TB = MLP_MAX_BATCH;              // 256
constexpr int SG = TB / TRAIN_NW;              // samples per group in the W2 product

struct __attribute__((aligned(16))) TrainShared {
  float P[MLP_NBLOCK + 1];
  float H1[TB * MLP_H];     // per-sample rows of 32, float4 chunks XOR-swizzled by row;
                            // the gradient G aliases it after the W2 product
  float DA2[TB * MLP_H];
  float H2[TB * MLP_H];     // the W2 partials (8 x 1024) alias it after use
  float DA1[TB * MLP_H];
  float XN[TB];
  float D3[TB];
  float A3P[2][TB];
  float SM[4][128];
  float WSUM[2][TRAIN_NW];
};

// chunk c (4 floats) of row s: rows of 8 chunks, chunk index XOR (s & 7) so that 64
// lanes storing one chunk of 64 consecutive rows, or reading 8 chunks of one row,
// touch distinct banks
__device__ inline float4* tchunk(float* A, int s, int c) {
  return reinterpret_cast<float4*>(A + s * MLP_H + 4 * (c ^ (s & 7)));
}
__device__ inline float telem(const float* A, int s, int i) { return A[s * MLP_H + 4 * ((i >> 2) ^ (s & 7)) + (i & 3)]; }

// Workgroup barrier that waits for this wave's LDS accesses only: global loads in
// flight (the next minibatch) stay in flight.  The empty asm statements keep the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_sync() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

__device__ inline float4 f4(float a, float b, float c, float d) {
  float4 v;
  v.x = a;
  v.y = b;
  v.z = c;
  v.w = d;
  return v;
}

// Forward and backward of sample (xv, tv) for this thread's sample slot (s < B
// valid), the gradient of the mean squared error over the B samples into G (which
// aliases H1) and the loss sum into *loss_sum (thread 128).  Starts after P is
// visible; ends with G visible to all threads.
__device__ float* batch_gradient(TrainShared& S, float xv, float tv, int B, float* loss_sum) {
  const int tid = threadIdx.x;
  const int s = tid & (TB - 1);
  const int hf = tid / TB;
  const int lane = tid & (WAVE - 1), w = tid / WAVE;
  const bool valid = s < B;
  const float* P = S.P;

  // F1: first layer (recomputed per chunk of 4 units), second layer (own 16 units),
  // partial output.  Each unit's sum runs over i = 0..31 in order.
  const float xn = __fmul_rn(__fsub_rn(xv, P[MLP_X0]), P[MLP_XS]);
  uint32_t m1 = 0;
  float a2[16];
#pragma unroll
  for (int jj = 0; jj < 16; jj++) a2[jj] = P[MLP_B2 + 16 * hf + jj];
#pragma nounroll
  for (int c = 0; c < 8; c++) {
    const float4 wv1 = *reinterpret_cast<const float4*>(P + MLP_W1 + 4 * c);
    const float4 bv1 = *reinterpret_cast<const float4*>(P + MLP_B1 + 4 * c);
    const float e0 = __fmaf_rn(wv1.x, xn, bv1.x), e1 = __fmaf_rn(wv1.y, xn, bv1.y),
                e2 = __fmaf_rn(wv1.z, xn, bv1.z), e3 = __fmaf_rn(wv1.w, xn, bv1.w);
    const float h0 = clamp01(e0), h1v = clamp01(e1), h2v = clamp01(e2), h3 = clamp01(e3);
    m1 |= (((e0 > 0.0f && e0 < 1.0f) ? 1u : 0u) | ((e1 > 0.0f && e1 < 1.0f) ? 2u : 0u) |
           ((e2 > 0.0f && e2 < 1.0f) ? 4u : 0u) | ((e3 > 0.0f && e3 < 1.0f) ? 8u : 0u))
          << (4 * c);
    if ((c >> 2) == hf) *tchunk(S.H1, s, c) = f4(h0, h1v, h2v, h3);
#pragma unroll
    for (int jj = 0; jj < 16; jj++) {
      const float4 wv = *reinterpret_cast<const float4*>(P + MLP_W2 + (16 * hf + jj) * MLP_H + 4 * c);
      float a = a2[jj];
      a = __fmaf_rn(wv.x, h0, a);
      a = __fmaf_rn(wv.y, h1v, a);
      a = __fmaf_rn(wv.z, h2v, a);
      a = __fmaf_rn(wv.w, h3, a);
      a2[jj] = a;
    }
  }
  uint32_t m2 = 0;
  float a3p = hf ? 0.0f : P[MLP_B3];
  {
    float h2[16];
#pragma unroll
    for (int jj = 0; jj < 16; jj++) {
      h2[jj] = clamp01(a2[jj]);
      m2 |= (a2[jj] > 0.0f && a2[jj] < 1.0f) ? (1u << jj) : 0u;
      a3p = __fmaf_rn(P[MLP_W3 + 16 * hf + jj], h2[jj], a3p);
    }
#pragma unroll
    for (int c = 0; c < 4; c++)
      *tchunk(S.H2, s, 4 * hf + c) = f4(h2[4 * c], h2[4 * c + 1], h2[4 * c + 2], h2[4 * c + 3]);
  }
  S.A3P[hf][s] = a3p;
  lds_sync();

  // F2: output, residual, output delta; second-layer deltas of own units
  const float a3 = __fadd_rn(S.A3P[0][s], S.A3P[1][s]);
  const float r = clamp01(a3) - tv;
  const float l = valid ? r * r : 0.0f;
  const float d3 = (valid && a3 > 0.0f && a3 < 1.0f) ? (2.0f / (float)B) * r : 0.0f;
  if (hf == 0) {
    S.XN[s] = xn;
    S.D3[s] = d3;
  }
  float da2[16];
#pragma unroll
  for (int jj = 0; jj < 16; jj++) da2[jj] = ((m2 >> jj) & 1u) ? d3 * P[MLP_W3 + 16 * hf + jj] : 0.0f;
#pragma unroll
  for (int c = 0; c < 4; c++)
    *tchunk(S.DA2, s, 4 * hf + c) = f4(da2[4 * c], da2[4 * c + 1], da2[4 * c + 2], da2[4 * c + 3]);
  {
    float sl = l, sd = d3;
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
      sl += __shfl_xor(sl, m);
      sd += __shfl_xor(sd, m);
    }
    if (lane == 0) {
      S.WSUM[0][w] = hf ? 0.0f : sl;
      S.WSUM[1][w] = hf ? 0.0f : sd;
    }
  }
  lds_sync();

  // F3: first-layer deltas of own units from all 32 second-layer deltas
  {
    float acc[16];
#pragma unroll
    for (int ii = 0; ii < 16; ii++) acc[ii] = 0.0f;
#pragma nounroll
    for (int c = 0; c < 8; c++) {
      const float4 dv = *tchunk(S.DA2, s, c);
      const float dj[4] = {dv.x, dv.y, dv.z, dv.w};
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const float4* wr = reinterpret_cast<const float4*>(P + MLP_W2 + (4 * c + e) * MLP_H + 16 * hf);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const float4 wv = wr[q];
          acc[4 * q] = fmaf(dj[e], wv.x, acc[4 * q]);
          acc[4 * q + 1] = fmaf(dj[e], wv.y, acc[4 * q + 1]);
          acc[4 * q + 2] = fmaf(dj[e], wv.z, acc[4 * q + 2]);
          acc[4 * q + 3] = fmaf(dj[e], wv.w, acc[4 * q + 3]);
        }
      }
    }
    const uint32_t mh = m1 >> (16 * hf);
#pragma unroll
    for (int c = 0; c < 4; c++) {
      float4 v;
      v.x = ((mh >> (4 * c)) & 1u) ? acc[4 * c] : 0.0f;
      v.y = ((mh >> (4 * c + 1)) & 1u) ? acc[4 * c + 1] : 0.0f;
      v.z = ((mh >> (4 * c + 2)) & 1u) ? acc[4 * c + 2] : 0.0f;
      v.w = ((mh >> (4 * c + 3)) & 1u) ? acc[4 * c + 3] : 0.0f;
      *tchunk(S.DA1, s, 4 * hf + c) = v;
    }
  }
  lds_sync();

  // G1: W2 gradient tile (rows 4jb.., columns 4ib..) over this wave's 32 samples, and
  // the vector gradients over a quarter of the samples
  const int jb = lane & 7, ib = lane >> 3;
  float g[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) g[a][b] = 0.0f;
#pragma unroll 8
  for (int q = 0; q < SG; q++) {
    const int s2 = w * SG + q;
    const float4 d = *tchunk(S.DA2, s2, jb);
    const float4 h = *tchunk(S.H1, s2, ib);
    const float dv[4] = {d.x, d.y, d.z, d.w};
    const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) g[a][b] = fmaf(dv[a], hv[b], g[a][b]);
  }
  // vector gradient o (0..31 w1, 32..63 b1, 64..95 b2, 96..127 w3) over quarter qq of
  // the samples, in sample order: each wave takes one kind (its 64 lanes: 32 outputs
  // times 2 quarters), so the loop has no divergent branch; x * 1 + sm is sm + x
  const int kind = w & 3;
  const int o = kind * 32 + (lane & 31), qq = (lane >> 5) + 2 * (w >> 2);
  const float* A = kind < 2 ? S.DA1 : (kind == 2 ? S.DA2 : S.H2);
  float sm = 0.0f;
#pragma unroll 16
  for (int q = 0; q < TB / 4; q++) {
    const int s2 = qq * (TB / 4) + q;
    const float mult = kind == 0 ? S.XN[s2] : (kind == 3 ? S.D3[s2] : 1.0f);
    sm = fmaf(telem(A, s2, o & 31), mult, sm);
  }
  lds_sync();

  // G2: partials to LDS (the W2 partials over H2, which is no longer read)
  float* red = S.H2;
#pragma unroll
  for (int a = 0; a < 4; a++)
    *reinterpret_cast<float4*>(red + w * (MLP_H * MLP_H) + (4 * jb + a) * MLP_H + 4 * ib) =
        f4(g[a][0], g[a][1], g[a][2], g[a][3]);
  S.SM[qq][o] = sm;
  lds_sync();

  // G3: reduce into G (over H1, no longer read)
  float* G = S.H1;
  for (int e = tid; e < MLP_H * MLP_H; e += TRAIN_P) {
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < TRAIN_NW; k++) v += red[k * (MLP_H * MLP_H) + e];
    G[MLP_W2 + e] = v;
  }
  if (tid < 128) {
    const float v = ((S.SM[0][tid] + S.SM[1][tid]) + S.SM[2][tid]) + S.SM[3][tid];
    const int dst = tid < 32 ? MLP_W1 + tid : tid < 64 ? MLP_B1 + (tid - 32) : tid < 96 ? MLP_B2 + (tid - 64)
                                                                                       : MLP_W3 + (tid - 96);
    G[dst] = v;
  } else if (tid == 128) {
    float sd = 0.0f, sl = 0.0f;
#pragma unroll
    for (int k = 0; k < TRAIN_NW; k++) {
      sd += S.WSUM[1][k];
      sl += S.WSUM[0][k];
    }
    G[MLP_B3] = sd;
    *loss_sum = sl;
  }
  lds_sync();
  return G;
}

__device__ inline void draw_sample(const TrainArgs& a, uint32_t step, int B, int s, float* xv, float* tv) {
  if (s < B && step <= a.steps) {
    const uint64_t draw = (uint64_t)(step - 1) * (uint64_t)B + (uint64_t)s;
    uint64_t idx;
    if (a.sequential) idx = draw % a.m;
    else idx = ((splitmix_at(a.seed, draw) >> 32) * a.m) >> 32;
    *xv = a.x[idx];
    *tv = a.t[idx];
  } else {
    *xv = 0.0f;
    *tv = 0.0f;
  }
}

// Adam (Kingma & Ba) with bias correction; step size decays linearly from lr to
// lr / 10; the first layer's parameters take 32x the step (their scale is 32x);
// weight matrices are projected onto w >= 0 after every step.
__global__ void __launch_bounds__(TRAIN_P) train_kernel(float* params, float* moments, TrainArgs a) {
  __shared__ TrainShared S;
  const int tid = threadIdx.x;
  for (int i = tid; i < MLP_NBLOCK; i += TRAIN_P) S.P[i] = params[i];
  constexpr int PER = (MLP_NPARAM + TRAIN_P - 1) / TRAIN_P;
  float mo[PER], ve[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = tid + q * TRAIN_P;
    mo[q] = i < MLP_NPARAM ? moments[i] : 0.0f;
    ve[q] = i < MLP_NPARAM ? moments[MLP_NPARAM + i] : 0.0f;
  }
  __syncthreads();
  const int B = (int)(a.batch < (uint32_t)TB ? a.batch : TB);
  const int s = tid & (TB - 1);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float b1t = 1.0f, b2t = 1.0f;
  float loss_sum = 0.0f;
  float xv, tv;
  draw_sample(a, 1, B, s, &xv, &tv);
  for (uint32_t step = 1; step <= a.steps; step++) {
    float xn_, tn_;
    draw_sample(a, step + 1, B, s, &xn_, &tn_);   // next minibatch, in flight meanwhile
    float* G = batch_gradient(S, xv, tv, B, &loss_sum);
    b1t *= b1;
    b2t *= b2;
    const float lr = a.lr * (1.0f - 0.9f * (float)(step - 1) / (float)(a.steps > 1 ? a.steps - 1 : 1));
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int i = tid + q * TRAIN_P;
      if (i < MLP_NPARAM) {
        const float g = G[i];
        mo[q] = b1 * mo[q] + (1.0f - b1) * g;
        ve[q] = b2 * ve[q] + (1.0f - b2) * g * g;
        const float mh = mo[q] / (1.0f - b1t), vh = ve[q] / (1.0f - b2t);
        const float mult = i < MLP_W2 ? 32.0f : 1.0f;
        float v = S.P[i] - lr * mult * mh / (sqrtf(vh) + eps);
        const bool nonneg = i < MLP_B1 || (i >= MLP_W2 && i < MLP_B2) || (i >= MLP_W3 && i < MLP_B3);
        if (nonneg) v = fmaxf(v, 0.0f);
        S.P[i] = v;
      }
    }
    lds_sync();
    xv = xn_;
    tv = tn_;
  }
  __syncthreads();
  for (int i = tid; i < MLP_NBLOCK; i += TRAIN_P) params[i] = S.P[i];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = tid + q * TRAIN_P;
    if (i < MLP_NPARAM) {
      moments[i] = mo[q];
      moments[MLP_NPARAM + i] = ve[q];
    }
  }
  if (tid == 128) moments[2 * MLP_NPARAM] = loss_sum / (float)(B > 0 ? B : 1);
}

// gradient of the mean squared error over m <= MLP_MAX_BATCH samples
__global__ void __launch_bounds__(TRAIN_P) gradient_kernel(const float* params, const float* x, const float* t,
                                                           uint32_t m, float* grad, float* loss) {
  __shared__ TrainShared S;
  const int tid = threadIdx.x;
  for (int i = tid; i < MLP_NBLOCK; i += TRAIN_P) S.P[i] = params[i];
  __syncthreads();
  const int B = (int)m;
  const int s = tid & (TB - 1);
  float loss_sum = 0.0f;
  const float* G = batch_gradient(S, s < B ? x[s] : 0.0f, s < B ? t[s] : 0.0f, B, &loss_sum);
  for (int i = tid; i < MLP_NPARAM; i += TRAIN_P) grad[i] = G[i];
  if (tid == 128) *loss = loss_sum / (float)B;
}

// ---- inference, thresholds, classification ----------------------------------------------

__global__ void forward_kernel(const float* params, const float* x, uint64_t m, float* y) {
  __shared__ float P[MLP_NBLOCK];
  for (int i = threadIdx.x; i < MLP_NBLOCK; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
    y[i] = mlp_forward(P, x[i]);
}

__global__ void buckets_kernel(const float* params, const uint64_t* keys, uint64_t n, int32_t* out) {
  __shared__ float P[MLP_NBLOCK];
  for (int i = threadIdx.x; i < MLP_NBLOCK; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = mlp_bucket(P, keys[i]);
}

// t_j = min{k : b(k) >= j} for j = 1..255, one wave per threshold: a 64-way search
// over all 64-bit keys (each round probes 64 evenly spaced keys of the interval that
// holds the answer, about 11 rounds); it relies on b being non-decreasing.
// nvalid = b(2^64 - 1): thresholds j > nvalid do not exist.
constexpr int THR_P = 256;
__global__ void __launch_bounds__(THR_P) thresholds_kernel(const float* params, uint64_t* thr, uint32_t* nvalid) {
  __shared__ float P[MLP_NBLOCK];
  for (int i = threadIdx.x; i < MLP_NBLOCK; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int j = blockIdx.x * (THR_P / WAVE) + threadIdx.x / WAVE + 1;
  const int top = mlp_bucket(P, ~0ull);
  if (j == 1 && lane == 0) *nvalid = (uint32_t)top;
  if (j >= NBUCKET) return;
  if (top < j) {
    if (lane == 0) thr[j - 1] = ~0ull;
    return;
  }
  uint64_t lo = 0, hi = ~0ull;   // the answer lies in [lo, hi]; b(hi) >= j
  while (lo < hi) {
    const uint64_t span = hi - lo;
    // probe l: lo + floor(span * l / 64) (exact), l = 0..63, all below hi
    const uint64_t pr = lo + (span >> 6) * (uint64_t)lane + (((span & 63) * (uint64_t)lane) >> 6);
    const uint64_t m = ballot(mlp_bucket(P, pr) >= j);
    if (m) {
      const int f = __builtin_ctzll(m);
      const uint64_t pf = (uint64_t)__shfl((long long)pr, f);
      const uint64_t pb = (uint64_t)__shfl((long long)pr, f > 0 ? f - 1 : 0);
      hi = pf;
      if (f > 0) lo = pb + 1;
    } else {
      lo = (uint64_t)__shfl((long long)pr, WAVE - 1) + 1;
    }
  }
  if (lane == 0) thr[j - 1] = lo;
}

__global__ void classify_kernel(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                                int32_t* out) {
  __shared__ uint64_t E[NBUCKET];
  tree_load(E, thr);
  __syncthreads();
  const int J = (int)*nvalid;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = classify(E, J, keys[i]);
}

// ---- 256-way partition ---------------------------------------------------------------------
//
// The input is cut into tiles of LEARN_TILE keys and the tiles into chunks of CHUNK_TILES
// consecutive tiles.  histogram_kernel counts every chunk's keys per bucket (chunk-major
// counts), scan_kernel turns each bucket's column into exclusive prefixes over the chunks,
// and scatter_kernel walks the tiles of a chunk in order in one workgroup, so that each
// bucket's keys of one chunk land as one contiguous stretch of the output, written from one
// XCD (partial cache lines only where a stretch begins or ends).

constexpr int LT_P = 256;
constexpr int HIST_TILE = 4096;             // keys a histogram workgroup counts per step
constexpr int LT_PER = HIST_TILE / LT_P;    // 16 keys per thread and step
constexpr int LT_NW = LT_P / WAVE;
static_assert((LEARN_TILE * CHUNK_TILES) % HIST_TILE == 0, "a chunk is whole histogram steps");
static_assert(LT_P == NBUCKET, "thread b of a workgroup owns bucket b");

// per-chunk bucket counts, chunk-major: hist[chunk * NBUCKET + b]
__global__ void __launch_bounds__(LT_P) histogram_kernel(const uint64_t* keys, uint64_t n, const uint64_t* thr,
                                                         const uint32_t* nvalid, uint32_t* hist, uint64_t nchunks) {
  __shared__ uint64_t E[NBUCKET];
  __shared__ uint32_t C[LT_NW][NBUCKET];     // one row per wave: fewer colliding LDS atomics
  tree_load(E, thr);
  const int J = (int)*nvalid;
  const int w = threadIdx.x / WAVE;
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    for (int i = threadIdx.x; i < LT_NW * NBUCKET; i += LT_P) (&C[0][0])[i] = 0;
    __syncthreads();
    // the chunk's keys in steps of HIST_TILE (the counts are per chunk, so the step
    // need not be the scatter's tile: 16 keys per thread keep seven waves per SIMD)
    constexpr uint64_t CHUNK = (uint64_t)LEARN_TILE * CHUNK_TILES;
    for (uint64_t base = ch * CHUNK; base < (ch + 1) * CHUNK; base += HIST_TILE) {
      if (base >= n) break;
      if (base + HIST_TILE <= n) {
        uint64_t k[LT_PER];
#pragma unroll
        for (int q = 0; q < LT_PER; q++) k[q] = keys[base + (uint64_t)q * LT_P + threadIdx.x];
        int bb[LT_PER];
#pragma unroll
        for (int q = 0; q < LT_PER; q++) bb[q] = classify(E, J, k[q]);
#pragma unroll
        for (int q = 0; q < LT_PER; q++) atomicAdd(&C[w][bb[q]], 1u);
      } else {
        for (int q = 0; q < LT_PER; q++) {
          const uint64_t i = base + (uint64_t)q * LT_P + threadIdx.x;
          if (i < n) atomicAdd(&C[w][classify(E, J, keys[i])], 1u);
        }
      }
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < LT_NW; r++) s += C[r][threadIdx.x];
    hist[ch * NBUCKET + threadIdx.x] = s;
    __syncthreads();
  }
}

// bucket b = blockIdx.x: the column hist[* NBUCKET + b] becomes its exclusive prefix over
// the chunks, in place; totals[b] = the column's sum.  Each thread takes a contiguous run
// of chunks (independent loads), then one workgroup scan of the run sums.
__global__ void __launch_bounds__(LT_P) scan_kernel(uint32_t* hist, uint64_t nchunks, uint64_t* totals) {
  __shared__ uint64_t W[LT_NW];
  const uint64_t b = blockIdx.x;
  const uint64_t per = (nchunks + LT_P - 1) / LT_P;
  const uint64_t c0 = min((uint64_t)threadIdx.x * per, nchunks), c1 = min(c0 + per, nchunks);
  uint64_t v = 0;
#pragma unroll 8
  for (uint64_t c = c0; c < c1; c++) v += hist[c * NBUCKET + b];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t o = (uint64_t)__shfl_up((long long)inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) W[w] = inc;
  __syncthreads();
  uint64_t run = inc - v;
  for (int k = 0; k < w; k++) run += W[k];
#pragma unroll 8
  for (uint64_t c = c0; c < c1; c++) {
    const uint32_t x = hist[c * NBUCKET + b];
    hist[c * NBUCKET + b] = (uint32_t)run;
    run += x;
  }
  if (threadIdx.x == LT_P - 1) totals[b] = run;
}

// bucket starts (offsets[0..256]) and a summary: [0] largest bucket, [1] buckets above
// overflow_factor * n / 256, [2] non-empty buckets; thread b takes bucket b
__global__ void __launch_bounds__(LT_P) offsets_kernel(const uint64_t* totals, uint64_t n, float overflow_factor,
                                                       int64_t* offsets, uint64_t* summary) {
  __shared__ uint64_t W[4][LT_NW];
  const int b = threadIdx.x, lane = b & (WAVE - 1), w = b / WAVE;
  const uint64_t v = totals[b];
  const double bound = (double)overflow_factor * (double)n / (double)NBUCKET;
  uint64_t inc = v, mx = v, over = (double)v > bound ? 1 : 0, nonempty = v ? 1 : 0;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t o = (uint64_t)__shfl_up((long long)inc, d);
    if (lane >= d) inc += o;
    const uint64_t om = (uint64_t)__shfl_xor((long long)mx, d);
    mx = om > mx ? om : mx;
    over += (uint64_t)__shfl_xor((long long)over, d);
    nonempty += (uint64_t)__shfl_xor((long long)nonempty, d);
  }
  if (lane == WAVE - 1) {
    W[0][w] = inc;
    W[1][w] = mx;
    W[2][w] = over;
    W[3][w] = nonempty;
  }
  __syncthreads();
  uint64_t before = 0;
  for (int k = 0; k < w; k++) before += W[0][k];
  offsets[b] = (int64_t)(before + inc - v);
  if (b == NBUCKET - 1) offsets[NBUCKET] = (int64_t)(before + inc);
  if (b == 0) {
    uint64_t m = 0, o = 0, ne = 0;
    for (int k = 0; k < LT_NW; k++) {
      m = W[1][k] > m ? W[1][k] : m;
      o += W[2][k];
      ne += W[3][k];
    }
    summary[0] = m;
    summary[1] = o;
    summary[2] = ne;
  }
}

// One chunk per workgroup iteration, its tiles in order.  Per tile: classify, rank inside
// the tile per bucket (LDS atomics), stage bucket-major in LDS, write each bucket's run of
// the tile to the bucket's running destination (offsets[b] + its keys in earlier chunks +
// its keys in earlier tiles of this chunk).  The next tile's loads are issued before the
// current tile is written out.  SC_P threads per workgroup; threads b < NBUCKET also own
// bucket b (its count, staged start and running destination).
#ifndef VQS_SCATTER_THREADS
#define VQS_SCATTER_THREADS 256
#endif
constexpr int SC_P = VQS_SCATTER_THREADS;
constexpr int SC_PER = LEARN_TILE / SC_P;   // keys per thread
static_assert(SC_P >= NBUCKET && SC_P % WAVE == 0 && LEARN_TILE % SC_P == 0, "scatter workgroup shape");

__global__ void __launch_bounds__(SC_P) scatter_kernel(const uint64_t* keys, uint64_t n, const uint64_t* thr,
                                                       const uint32_t* nvalid, const uint32_t* hist,
                                                       uint64_t nchunks, const int64_t* offsets, uint64_t* out) {
  __shared__ uint64_t E[NBUCKET];
  __shared__ uint32_t C[NBUCKET];            // the tile's bucket counts; zero between tiles
  __shared__ uint32_t LO[NBUCKET];           // start of bucket b in the staged tile
  __shared__ uint64_t DL[NBUCKET];           // destination of staged slot s of bucket b: DL[b] + s
  __shared__ uint64_t stage[LEARN_TILE];
  __shared__ uint8_t bid[LEARN_TILE];
  __shared__ uint32_t W[NBUCKET / WAVE];
  const bool own = threadIdx.x < NBUCKET;
  tree_load(E, thr);
  if (own) C[threadIdx.x] = 0;
  const int J = (int)*nvalid;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const uint64_t ntiles = (n + LEARN_TILE - 1) / LEARN_TILE;
  uint64_t k[SC_PER];
  auto load = [&](uint64_t tile) {
    const uint64_t base = tile * LEARN_TILE;
    if (base + LEARN_TILE <= n) {
#pragma unroll
      for (int q = 0; q < SC_PER; q++) k[q] = keys[base + (uint64_t)q * SC_P + threadIdx.x];
    } else {
#pragma unroll
      for (int q = 0; q < SC_PER; q++) {
        const uint64_t i = base + (uint64_t)q * SC_P + threadIdx.x;
        k[q] = i < n ? keys[i] : 0;
      }
    }
  };
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    // thread b < NBUCKET alone reads and writes dst (its bucket's running destination)
    uint64_t dst = own ? (uint64_t)offsets[threadIdx.x] + hist[ch * NBUCKET + threadIdx.x] : 0;
    const uint64_t t0 = ch * CHUNK_TILES, t1 = min(t0 + CHUNK_TILES, ntiles);
    load(t0);
    __syncthreads();
    for (uint64_t tile = t0; tile < t1; tile++) {
      const uint32_t cnt = (uint32_t)min((uint64_t)LEARN_TILE, n - tile * LEARN_TILE);
      int bb[SC_PER];
      uint32_t r[SC_PER];
#pragma unroll
      for (int q = 0; q < SC_PER; q++) bb[q] = classify(E, J, k[q]);
      if (cnt == LEARN_TILE) {
#pragma unroll
        for (int q = 0; q < SC_PER; q++) r[q] = atomicAdd(&C[bb[q]], 1u);
      } else {
#pragma unroll
        for (int q = 0; q < SC_PER; q++)
          r[q] = (uint32_t)(q * SC_P + threadIdx.x) < cnt ? atomicAdd(&C[bb[q]], 1u) : 0u;
      }
      __syncthreads();
      {  // exclusive scan of the tile's bucket counts; thread b owns C[b] from here on
        const uint32_t v = own ? C[threadIdx.x] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
          const uint32_t o = (uint32_t)__shfl_up((int)inc, d);
          if (lane >= d) inc += o;
        }
        if (own && lane == WAVE - 1) W[w] = inc;
        __syncthreads();
        if (own) {
          uint32_t lo = inc - v;
          for (int kk = 0; kk < w; kk++) lo += W[kk];
          LO[threadIdx.x] = lo;
          DL[threadIdx.x] = dst - lo;
          dst += v;
          C[threadIdx.x] = 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SC_PER; q++) {
        if ((uint32_t)(q * SC_P + threadIdx.x) < cnt) {
          const uint32_t pos = LO[bb[q]] + r[q];
          stage[pos] = k[q];
          bid[pos] = (uint8_t)bb[q];
        }
      }
      __syncthreads();
      if (tile + 1 < t1) load(tile + 1);
      // destinations lie below n by construction (the histogram counted these very keys);
      // the clamp keeps every store inside the output even for an input changed in between
      if (cnt == LEARN_TILE) {
#pragma unroll
        for (int q = 0; q < SC_PER; q++) {
          const uint32_t s = q * SC_P + threadIdx.x;
          out[min(DL[bid[s]] + s, n - 1)] = stage[s];
        }
      } else {
        for (uint32_t s = threadIdx.x; s < cnt; s += SC_P) out[min(DL[bid[s]] + s, n - 1)] = stage[s];
      }
      __syncthreads();
    }
  }
}

int grid_for(uint64_t work, int per, int cap) {
  uint64_t g = (work + per - 1) / per;
  if (g < 1) g = 1;
  if (g > (uint64_t)cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_sample(const uint64_t* keys, uint64_t n, uint64_t* sample, uint64_t chunks, uint64_t seed,
                         hipStream_t s) {
  hipLaunchKernelGGL(sample_kernel, dim3(grid_for(chunks * 8, 256, 8192)), dim3(256), 0, s, keys, n, sample, chunks, seed);
  return hipGetLastError();
}

hipError_t launch_targets(const uint64_t* sorted, uint64_t m, float* x, float* t, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3(grid_for(m, 256, 8192)), dim3(256), 0, s, sorted, m, x, t);
  return hipGetLastError();
}

hipError_t launch_init(float* params, uint64_t seed, const float* x, uint64_t m, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(256), 0, s, params, seed, x, m);
  return hipGetLastError();
}

hipError_t launch_train(float* params, float* moments, const TrainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(train_kernel, dim3(1), dim3(TRAIN_P), 0, s, params, moments, a);
  return hipGetLastError();
}

hipError_t launch_gradient(const float* params, const float* x, const float* t, uint32_t m, float* grad, float* loss,
                           hipStream_t s) {
  hipLaunchKernelGGL(gradient_kernel, dim3(1), dim3(TRAIN_P), 0, s, params, x, t, m, grad, loss);
  return hipGetLastError();
}

hipError_t launch_forward(const float* params, const float* x, uint64_t m, float* y, hipStream_t s) {
  hipLaunchKernelGGL(forward_kernel, dim3(grid_for(m, 256, 4096)), dim3(256), 0, s, params, x, m, y);
  return hipGetLastError();
}

hipError_t launch_buckets(const float* params, const uint64_t* keys, uint64_t n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(buckets_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, params, keys, n, out);
  return hipGetLastError();
}

hipError_t launch_thresholds(const float* params, uint64_t* thr, uint32_t* nvalid, hipStream_t s) {
  hipLaunchKernelGGL(thresholds_kernel, dim3(NBUCKET / (THR_P / WAVE)), dim3(THR_P), 0, s, params, thr, nvalid);
  return hipGetLastError();
}

hipError_t launch_classify(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid, int32_t* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(classify_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, keys, n, thr, nvalid, out);
  return hipGetLastError();
}

hipError_t launch_histogram(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                            uint32_t* hist, uint64_t nchunks, hipStream_t s) {
  hipLaunchKernelGGL(histogram_kernel, dim3(grid_for(nchunks, 1, 1 << 20)), dim3(LT_P), 0, s, keys, n, thr, nvalid,
                     hist, nchunks);
  return hipGetLastError();
}

hipError_t launch_scan(uint32_t* hist, uint64_t nchunks, uint64_t* totals, hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(NBUCKET), dim3(LT_P), 0, s, hist, nchunks, totals);
  return hipGetLastError();
}

hipError_t launch_offsets(const uint64_t* totals, uint64_t n, float overflow_factor, int64_t* offsets,
                          uint64_t* summary, hipStream_t s) {
  hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(LT_P), 0, s, totals, n, overflow_factor, offsets, summary);
  return hipGetLastError();
}

hipError_t launch_scatter(const uint64_t* keys, uint64_t n, const uint64_t* thr, const uint32_t* nvalid,
                          const uint32_t* hist, uint64_t nchunks, const int64_t* offsets, uint64_t* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(nchunks, 1, 1 << 20)), dim3(SC_P), 0, s, keys, n, thr, nvalid,
                     hist, nchunks, offsets, out);
  return hipGetLastError();
}

}  // namespace vqs
