/*
 * mlp_oracle.c -- scalar FP32 reference of the learned bucket map.
 *
 * TEST INFRASTRUCTURE ONLY (see vqs_oracle.c).  The GPU library does not use it.
 *
 * The model is a 1 -> 32 -> 32 -> 1 perceptron with clamp-to-[0,1] activations and
 * non-negative weights, read as an approximation of the key distribution's CDF;
 * bucket(k) = min(255, floor(256 * y(x(k)))).  Every FP32 operation below is one
 * IEEE operation with round-to-nearest (compiled with -ffp-contract=off, fused
 * multiply-adds written as fmaf), in a fixed order, so a device implementation that
 * performs the same operations in the same order produces bit-identical bucket ids.
 *
 * Parameter block (floats): w1[32] b1[32] W2[32][32] (row j = hidden unit j of the
 * second layer, column i = first-layer unit i) b2[32] w3[32] b3, then the input
 * normalisation x0, xs (x' = (x - x0) * xs).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define H 32
#define P_W1 0
#define P_B1 (P_W1 + H)
#define P_W2 (P_B1 + H)
#define P_B2 (P_W2 + H * H)
#define P_W3 (P_B2 + H)
#define P_B3 (P_W3 + H)
#define P_X0 (P_B3 + 1)
#define P_XS (P_X0 + 1)

static float clamp01(float a) { return fminf(fmaxf(a, 0.0f), 1.0f); }

/* Monotone input map: the key rounded to the nearest float, whose bit pattern,
 * read as an unsigned integer, is converted to float and scaled by 2^-31. */
static float key_to_x_u64(uint64_t k) {
    float f = (float)k;
    uint32_t bits;
    memcpy(&bits, &f, 4);
    return (float)bits * 0x1p-31f;
}

static float forward(const float* p, float x) {
    float h1[H];
    const float xn = (x - p[P_X0]) * p[P_XS];
    for (int i = 0; i < H; i++) h1[i] = clamp01(fmaf(p[P_W1 + i], xn, p[P_B1 + i]));
    float y = p[P_B3];
    for (int j = 0; j < H; j++) {
        float a = p[P_B2 + j];
        for (int i = 0; i < H; i++) a = fmaf(p[P_W2 + j * H + i], h1[i], a);
        y = fmaf(p[P_W3 + j], clamp01(a), y);
    }
    return clamp01(y);
}

static int bucket_of(float y, int nbuckets) {
    int b = (int)(y * (float)nbuckets);      /* y in [0,1]: exact scaling by a power of two */
    return b < nbuckets - 1 ? b : nbuckets - 1;
}

void vqo_key_to_x_u64(const uint64_t* keys, uint64_t n, float* x) {
    for (uint64_t i = 0; i < n; i++) x[i] = key_to_x_u64(keys[i]);
}

void vqo_mlp_forward_f32(const float* params, const float* x, uint64_t n, float* y) {
    for (uint64_t i = 0; i < n; i++) y[i] = forward(params, x[i]);
}

void vqo_mlp_bucket_u64(const float* params, const uint64_t* keys, uint64_t n, int nbuckets,
                        int32_t* out) {
    for (uint64_t i = 0; i < n; i++) out[i] = bucket_of(forward(params, key_to_x_u64(keys[i])), nbuckets);
}
