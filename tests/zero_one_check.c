/* zero_one_check.c -- exhaustive 0-1 check of a comparator network, bitsliced.
 *
 * Test helper: it evaluates a given list of compare-and-exchange modules (built by
 * the oracle) on every 0-1 input and holds no part of the sort's arithmetic.  Input
 * number i = 64 * w + b sits in bit b of word w; wire k < nfree carries bit k of i,
 * the other wires carry the padding value 1.  A module (a, b) leaves min (AND) on a
 * and max (OR) on b.  The output, read through `order`, must be non-decreasing for
 * every input. */
#include <stdint.h>

#define MAXW 1024

/* Returns -1 when all 2^nfree inputs come out sorted, else the first failing word. */
int64_t zero_one_check(const uint32_t* pairs, int nmod, const uint32_t* order, int cells, int nfree) {
    const uint64_t words = nfree >= 6 ? (1ull << (nfree - 6)) : 1;
    uint64_t pat[6];
    for (int k = 0; k < 6; k++) {
        pat[k] = 0;
        for (int b = 0; b < 64; b++)
            if ((b >> k) & 1) pat[k] |= 1ull << b;
    }
    uint64_t w[MAXW];
    for (uint64_t word = 0; word < words; word++) {
        for (int k = 0; k < cells; k++) {
            if (k >= nfree) w[k] = ~0ull;
            else if (k < 6) w[k] = pat[k];
            else w[k] = ((word >> (k - 6)) & 1) ? ~0ull : 0ull;
        }
        if (nfree < 6) {   /* only the first 2^nfree lanes are inputs */
            const uint64_t live = (1ull << (1u << nfree)) - 1;
            for (int k = 0; k < cells; k++) w[k] &= live;
            (void)live;
        }
        for (int m = 0; m < nmod; m++) {
            const uint32_t a = pairs[2 * m], b = pairs[2 * m + 1];
            const uint64_t lo = w[a] & w[b];
            w[b] |= w[a];
            w[a] = lo;
        }
        uint64_t bad = 0;
        for (int k = 0; k + 1 < cells; k++) bad |= w[order[k]] & ~w[order[k + 1]];
        if (bad) return (int64_t)word;
    }
    return -1;
}
