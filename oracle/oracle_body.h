/*
 * oracle_body.h -- type-generic body of the scalar CPU oracle.
 *
 * TEST INFRASTRUCTURE: only tests/, the smoke check and the CPU-baseline leg of
 * bench.py use the oracle.  It shares no code with the GPU library.
 *
 * Included once per key type by vqs_oracle.c with these macros defined:
 *   KT            the C key type
 *   SFX(name)     pastes a per-type suffix onto a name
 *   KLESS(a, b)   the natural strict order of KT (ascending)
 *   KMAXV, KMINV  the last / first value of KT in ascending order (padding)
 *   KW            keys per 64-byte sampling chunk (64 / sizeof(KT))
 *
 * Every routine follows one step of the paper's method:
 *   Sec. 2 / Alg. 1    Recurse (partition, degenerate handling, base case, tail calls)
 *   Sec. 2.1           Partition (keys not after the pivot go left): the plain
 *                      out-of-place split, or the paper's in-place bidirectional scan
 *   Sec. 2.2           ChoosePivot (nine random 64-byte chunks, medians of three),
 *                      depth limit 2*log2(n)+4 with Heapsort as the fallback
 *   Sec. 2.3, Sec. 3   BaseCase (16-row matrix, Green's 16-input column network,
 *                      bitonic merges of adjacent sorted column groups)
 *   Sec. 2.4           sort order (ascending / descending) via a single "before" relation
 */

/* "a is before b" in the requested sort order (Sec. 2.4: OrderAscending /
 * OrderDescending define Compare; descending is the mirrored relation). */
static inline int SFX(before)(KT a, KT b, int asc) { return asc ? KLESS(a, b) : KLESS(b, a); }

/* Compare-and-exchange module (Sec. 3): afterwards *a is not after *b. */
static inline void SFX(cex)(KT* a, KT* b, int asc) {
    if (SFX(before)(*b, *a, asc)) { KT t = *a; *a = *b; *b = t; }
}

/* Median of three with the network (0,2) (0,1) (1,2) of Sec. 2.2; element 1 is
 * the median afterwards. */
static KT SFX(med3)(KT x0, KT x1, KT x2, int asc) {
    SFX(cex)(&x0, &x2, asc);
    SFX(cex)(&x0, &x1, asc);
    SFX(cex)(&x1, &x2, asc);
    return x1;
}

/* ChoosePivot (Sec. 2.2).  Nine chunks of KW keys (64 bytes) are taken at random
 * chunk-aligned offsets relative to the range start; lanewise medians of three over
 * chunk groups (0,1,2), (3,4,5), (6,7,8) give 3*KW medians.  These are reduced by
 * medians of three: first whole "vectors" of KW lanes three at a time, then single
 * consecutive triples, dropping the 0..2 leftovers, until fewer than three remain.
 * The first remaining median is the pivot. */
static KT SFX(choose_pivot)(const KT* keys, uint64_t b, uint64_t e, const vqo_params* p) {
    const int asc = p->ascending;
    const uint64_t W = KW;
    const uint64_t nchunks = (e - b) / W;      /* whole chunks; the tail is never sampled */
    uint32_t u[10];
    range_draws(p, b, e, u);                   /* five 64-bit draws -> ten 32-bit halves */
    const KT* chunk[9];
    for (int i = 0; i < 9; i++) {
        uint64_t off = multiply_shift_offset(u[i], nchunks);
        chunk[i] = keys + b + off * W;
    }
    KT bufA[3 * KW], bufB[3 * KW];
    KT* cur = bufA;
    KT* nxt = bufB;
    for (uint64_t g = 0; g < 3; g++)
        for (uint64_t j = 0; j < W; j++)
            cur[g * W + j] = SFX(med3)(chunk[3 * g][j], chunk[3 * g + 1][j], chunk[3 * g + 2][j], asc);
    uint64_t m = 3 * W;
    while (m >= 3) {
        uint64_t i = 0, o = 0;
        while (i + 3 * W <= m) {              /* whole vectors, lanewise */
            for (uint64_t j = 0; j < W; j++)
                nxt[o++] = SFX(med3)(cur[i + j], cur[i + W + j], cur[i + 2 * W + j], asc);
            i += 3 * W;
        }
        while (i + 3 <= m) {                  /* single elements */
            nxt[o++] = SFX(med3)(cur[i], cur[i + 1], cur[i + 2], asc);
            i += 3;
        }
        KT* t = cur; cur = nxt; nxt = t;
        m = o;
    }
    return cur[0];
}

/* Partition (Sec. 2.1): keys not after the pivot move before all others; returns
 * the index of the first key of the right side.  Written as a plain out-of-place
 * split: a single scan places left keys from the front in input order and right
 * keys from the back (so in reverse input order); the buffer is copied back. */
static uint64_t SFX(partition)(KT* keys, KT* tmp, uint64_t b, uint64_t e, KT pivot, int asc) {
    uint64_t l = b, r = e;
    for (uint64_t i = b; i < e; i++) {
        KT k = keys[i];
        if (!SFX(before)(pivot, k, asc)) tmp[l++] = k;
        else tmp[--r] = k;
    }
    memcpy(keys + b, tmp + b, (e - b) * sizeof(KT));
    return l;
}

/* In-place Partition (Sec. 2.1): the bidirectional scan, taken with a vector of
 * IP_LANES keys and IP_UNROLL vectors per loop iteration (one "block").  Only
 * O(block) keys are held outside the array.
 *
 *  1. A range of fewer than two blocks, or else its first n mod IP_BLOCK keys, goes
 *     through the small loop: keys not after the pivot are compress-stored in place
 *     from the front, the others collected in order in a buffer.  The range's last
 *     keys, as many as the buffer holds, then move in order into the gap behind the
 *     left keys, and the buffer is stored at the end of the range.
 *  2. The rest of the range, whole blocks (at least two), is the main loop's input.
 *     Its first and last blocks are held back (read first, partitioned last).  Each
 *     iteration loads the next unread block from the side whose capacity (distance
 *     between read and write position) is smaller, the left side on a tie, and
 *     partitions its vectors in address order: a vector's left keys are stored at
 *     writeL in lane order, writeR moves down by the number of its right keys, which
 *     are stored from writeR in lane order.
 *  3. The two held-back blocks, first then last, are partitioned the same way.  The
 *     write positions then meet at the bound.
 *
 * Stores write exactly the valid lanes, so the paper's last-vector adjustment for a
 * blended store that could touch memory past the range does not apply. */
#ifndef IP_LANES
#define IP_LANES 64
#define IP_UNROLL 4
#define IP_BLOCK (IP_LANES * IP_UNROLL)
#endif

/* One vector's CompressStores (step 2 above). */
static void SFX(ip_vector)(KT* keys, const KT* v, KT pivot, int asc, uint64_t* wl, uint64_t* wr) {
    KT right[IP_LANES];
    uint64_t nr = 0;
    for (uint64_t x = 0; x < IP_LANES; x++) {
        if (!SFX(before)(pivot, v[x], asc)) keys[(*wl)++] = v[x];
        else right[nr++] = v[x];
    }
    *wr -= nr;
    memcpy(keys + *wr, right, nr * sizeof(KT));
}

static uint64_t SFX(partition_inplace)(KT* keys, uint64_t b, uint64_t e, KT pivot, int asc) {
    const uint64_t n = e - b;
    const uint64_t nrem = n < 2 * IP_BLOCK ? n : n % IP_BLOCK;
    KT buf[IP_BLOCK], first[IP_BLOCK], last[IP_BLOCK], blk[IP_BLOCK];
    /* 1. the small loop */
    uint64_t left = b, nbuf = 0;
    for (uint64_t i = b; i < b + nrem; i++) {
        const KT k = keys[i];
        if (!SFX(before)(pivot, k, asc)) keys[left++] = k;
        else buf[nbuf++] = k;
    }
    const uint64_t right = e - nbuf;
    memmove(keys + left, keys + right, nbuf * sizeof(KT));
    memcpy(keys + right, buf, nbuf * sizeof(KT));
    if (nrem == n) return left;
    /* 2. the main loop on [left, right) */
    memcpy(first, keys + left, sizeof(first));
    memcpy(last, keys + right - IP_BLOCK, sizeof(last));
    uint64_t readL = left + IP_BLOCK, readR = right - IP_BLOCK;
    uint64_t wl = left, wr = right;
    while (readL < readR) {
        if (readL - wl <= wr - readR) {
            memcpy(blk, keys + readL, sizeof(blk));
            readL += IP_BLOCK;
        } else {
            readR -= IP_BLOCK;
            memcpy(blk, keys + readR, sizeof(blk));
        }
        for (int v = 0; v < IP_UNROLL; v++) SFX(ip_vector)(keys, blk + v * IP_LANES, pivot, asc, &wl, &wr);
    }
    /* 3. the held-back blocks */
    for (int v = 0; v < IP_UNROLL; v++) SFX(ip_vector)(keys, first + v * IP_LANES, pivot, asc, &wl, &wr);
    for (int v = 0; v < IP_UNROLL; v++) SFX(ip_vector)(keys, last + v * IP_LANES, pivot, asc, &wl, &wr);
    return wl;
}

/* ScanMinMax (Alg. 1): first and last key of the range in sort order. */
static void SFX(minmax)(const KT* keys, uint64_t b, uint64_t e, int asc, KT* first, KT* last) {
    KT f = keys[b], l = keys[b];
    for (uint64_t i = b + 1; i < e; i++) {
        if (SFX(before)(keys[i], f, asc)) f = keys[i];
        if (SFX(before)(l, keys[i], asc)) l = keys[i];
    }
    *first = f;
    *last = l;
}

/* Textbook Heapsort (the depth-limit fallback of Sec. 2.2). */
static void SFX(sift_down)(KT* a, uint64_t i, uint64_t n, int asc) {
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= n) return;
        if (c + 1 < n && SFX(before)(a[c], a[c + 1], asc)) c++;
        if (!SFX(before)(a[i], a[c], asc)) return;
        KT t = a[i]; a[i] = a[c]; a[c] = t;
        i = c;
    }
}

static void SFX(heapsort)(KT* a, uint64_t n, int asc) {
    if (n < 2) return;
    for (uint64_t i = n / 2; i-- > 0;) SFX(sift_down)(a, i, n, asc);
    for (uint64_t end = n - 1; end > 0; end--) {
        KT t = a[0]; a[0] = a[end]; a[end] = t;
        SFX(sift_down)(a, 0, end, asc);
    }
}

/* BaseCase (Sec. 2.3 and Sec. 3).  The n <= 16*c keys are copied into a buffer
 * viewed as a row-major matrix of 16 rows and c columns (c the smallest power of
 * two with 16*c >= n), padded with the last value in sort order so the padding
 * stays in place.  Then the network of basecase_network runs on the cells: each
 * column is sorted with Green's 60-module network, then adjacent sorted groups of w
 * columns are merged into groups of 2w columns with the bitonic merge network (flip
 * stage, then half-cleaners) until one group remains; a group's sorted sequence is
 * its elements in row-major order.  The keys leave in the network's output order. */
static void SFX(basecase)(KT* keys, uint64_t n, int asc) {
    if (n < 2) return;
    int lc = 0;
    while ((16ull << lc) < n) lc++;
    const bc_net* net = &BC_NET[lc];
    KT buf[BC_MAX_CELLS];
    memcpy(buf, keys, n * sizeof(KT));
    const KT last = asc ? KMAXV : KMINV;
    for (uint64_t i = n; i < net->cells; i++) buf[i] = last;
    for (int m = 0; m < net->nmod; m++) SFX(cex)(&buf[net->pairs[m][0]], &buf[net->pairs[m][1]], asc);
    for (uint64_t k = 0; k < n; k++) keys[k] = buf[net->order[k]];
}

/* Recurse (Alg. 1).  depth counts nested Recurse calls (the first call is 1); a
 * call deeper than the limit Heapsorts its range instead. */
static void SFX(recurse)(KT* keys, KT* tmp, uint64_t b, uint64_t e, KT pivot, uint64_t depth,
                         const vqo_params* p, vqo_stats* st) {
    if (depth > st->depth_limit_used) {
        SFX(heapsort)(keys + b, e - b, p->ascending);
        st->heapsorts++;
        st->heapsort_keys += e - b;
        return;
    }
    if (depth > st->max_depth) st->max_depth = depth;
    const uint64_t bound = p->inplace ? SFX(partition_inplace)(keys, b, e, pivot, p->ascending)
                                      : SFX(partition)(keys, tmp, b, e, pivot, p->ascending);
    st->partitions++;
    st->keys_partitioned += e - b;
    if (bound == e) {                               /* degenerate: right side empty */
        KT first, last;
        st->degenerate++;
        SFX(minmax)(keys, b, e, p->ascending, &first, &last);
        if (!SFX(before)(first, last, p->ascending)) {  /* all keys equal */
            st->all_equal++;
            return;
        }
        SFX(recurse)(keys, tmp, b, e, first, depth + 1, p, st);
        return;
    }
    if (bound - b <= p->nb) {
        SFX(basecase)(keys + b, bound - b, p->ascending);
        st->basecases++;
    } else {
        KT next = SFX(choose_pivot)(keys, b, bound, p);
        SFX(recurse)(keys, tmp, b, bound, next, depth + 1, p, st);
    }
    if (e - bound <= p->nb) {
        SFX(basecase)(keys + bound, e - bound, p->ascending);
        st->basecases++;
    } else {
        KT next = SFX(choose_pivot)(keys, bound, e, p);
        SFX(recurse)(keys, tmp, bound, e, next, depth + 1, p, st);
    }
}

/* Sort the range [b, e) of keys (positions are absolute, they seed the sampler). */
static void SFX(sort_range)(KT* keys, KT* tmp, uint64_t b, uint64_t e, const vqo_params* p,
                            vqo_stats* st) {
    const uint64_t n = e - b;
    if (n <= p->nb) {
        SFX(basecase)(keys + b, n, p->ascending);
        if (n > 0) st->basecases++;
        return;
    }
    st->depth_limit_used = p->depth_limit >= 0 ? (uint64_t)p->depth_limit : default_depth_limit(n);
    KT pivot = SFX(choose_pivot)(keys, b, e, p);
    SFX(recurse)(keys, tmp, b, e, pivot, 1, p, st);
}
