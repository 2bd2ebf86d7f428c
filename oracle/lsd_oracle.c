/*
 * lsd_oracle.c -- CPU oracle for the stable LSD radix sort.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * library under paper_1008_2849_amd/ never includes, links or calls it, and
 * it shares no code with that library.
 *
 * What it computes, from Wassenberg & Sanders, "Faster Radix Sort via Virtual
 * Memory and Write-Combining" (arXiv:1008.2849):
 *
 *   - Section 3 (naive counting sort): build the histogram of the N keys;
 *     an exclusive prefix sum of it gives the first output slot of every key
 *     value; then each item is written at its key's slot, and that slot is
 *     incremented.  Here the "key" of a pass is one digit of the 32-bit key.
 *   - Section 4 (LSD radix sort): D-bit digits of the K-bit keys are taken
 *     from the least significant one upward; each pass partitions all items
 *     by the current digit and preserves the order of items with equal
 *     digits (stability), so after the last pass the items are in ascending
 *     key order with equal keys in input order.
 *   - Items are a 32-bit key with an optional 32-bit value (abstract,
 *     Section 1); values travel with their keys.
 *
 * Plain choices, made on purpose: one thread, no SIMD, no pass skipping,
 * 64-bit counters, a fresh output array per pass (out of place, as the
 * paper's passes are), and the items visited in increasing input order in
 * every scatter.
 *
 * Digit widths are given per pass, least significant first, and must sum
 * to 32; each width is 1..16 (a wider digit would need a 2^width counter
 * array, which a plain oracle has no reason to allocate).
 *
 * Return codes: 0 = ok, -1 = invalid arguments, -2 = out of host memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Digit of a key: bits [shift, shift + width) (Section 4, digit extraction). */
static uint32_t digit_of(uint32_t key, unsigned shift, unsigned width)
{
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 5
    /* planted mistake: the mask drops the digit's top bit */
    return (key >> shift) & ((1u << (width - 1)) - 1u);
#elif defined(ORACLE_MUTANT) && ORACLE_MUTANT == 6
    /* planted mistake: keys compared as signed (sign bit flipped) */
    return ((key ^ 0x80000000u) >> shift) & ((1u << width) - 1u);
#else
    return (key >> shift) & ((1u << width) - 1u);
#endif
}

static int widths_ok(const unsigned *widths, unsigned npasses)
{
    unsigned total = 0, p;
    if (widths == NULL || npasses == 0 || npasses > 32)
        return 0;
    for (p = 0; p < npasses; ++p) {
        if (widths[p] < 1 || widths[p] > 16)
            return 0;
        total += widths[p];
    }
    return total == 32;
}

/*
 * Histogram of one digit over n keys (Section 3, first step of counting
 * sort).  hist must hold 2^width counters; it is overwritten.
 */
int oracle_digit_histogram(const uint32_t *keys, uint64_t n, unsigned shift,
                           unsigned width, uint64_t *hist)
{
    uint64_t i, buckets;
    if (width < 1 || width > 16 || shift + width > 32 || hist == NULL ||
        (keys == NULL && n > 0))
        return ORACLE_EINVAL;
    buckets = (uint64_t)1 << width;
    for (i = 0; i < buckets; ++i)
        hist[i] = 0;
    for (i = 0; i < n; ++i)
        hist[digit_of(keys[i], shift, width)] += 1;
    return ORACLE_OK;
}

/*
 * One counting-sort pass (Section 3, naive algorithm), out of place:
 * histogram, exclusive prefix sum, then every item in increasing input
 * order written at its digit's next slot.  vin/vout are both NULL for a
 * keys-only pass.
 */
int oracle_counting_pass(const uint32_t *kin, const uint32_t *vin,
                         uint32_t *kout, uint32_t *vout, uint64_t n,
                         unsigned shift, unsigned width)
{
    uint64_t buckets, d, i, running;
    uint64_t *next;
    int rc;
    if ((vin == NULL) != (vout == NULL))
        return ORACLE_EINVAL;
    if (n > 0 && (kin == NULL || kout == NULL))
        return ORACLE_EINVAL;
    if (width < 1 || width > 16 || shift + width > 32)
        return ORACLE_EINVAL;
    buckets = (uint64_t)1 << width;
    next = (uint64_t *)malloc(buckets * sizeof(uint64_t));
    if (next == NULL)
        return ORACLE_ENOMEM;

    /* step 1: histogram of the digit */
    rc = oracle_digit_histogram(kin, n, shift, width, next);
    if (rc != ORACLE_OK) {
        free(next);
        return rc;
    }

    /* step 2: exclusive prefix sum -> first output slot of each digit */
    running = 0;
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 2
    /* planted mistake: the sum runs over the digits in descending order */
    for (d = buckets; d-- > 0;) {
        uint64_t count = next[d];
        next[d] = running;
        running += count;
    }
#else
    for (d = 0; d < buckets; ++d) {
        uint64_t count = next[d];
        next[d] = running;
        running += count;
    }
#endif

    /* step 3: scatter; each item goes to its digit's slot, then the slot
     * moves on by one, so equal digits keep their input order */
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 1
    /* planted mistake: items visited in decreasing order while the slots
     * still move forward, which reverses every run of equal digits */
    for (i = n; i-- > 0;) {
        uint32_t dd = digit_of(kin[i], shift, width);
        kout[next[dd]] = kin[i];
        if (vin != NULL)
            vout[next[dd]] = vin[i];
        next[dd] += 1;
    }
#else
    for (i = 0; i < n; ++i) {
        uint32_t dd = digit_of(kin[i], shift, width);
        uint64_t slot = next[dd];
        kout[slot] = kin[i];
        if (vin != NULL) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 4
            /* planted mistake: values stay in input order */
            vout[i] = vin[i];
#else
            vout[slot] = vin[i];
#endif
        }
        next[dd] = slot + 1;
    }
#endif
    free(next);
    return ORACLE_OK;
}

/*
 * Full LSD radix sort (Section 4): passes over the digits from the least
 * significant upward, each a stable counting-sort pass.  The result
 * replaces keys[] (and vals[] when not NULL).
 */
int oracle_lsd_sort(uint32_t *keys, uint32_t *vals, uint64_t n,
                    const unsigned *widths, unsigned npasses)
{
    uint32_t *ka, *kb, *va = NULL, *vb = NULL, *tmp;
    unsigned p, shift = 0, last = npasses;
    int rc = ORACLE_OK;
    if (!widths_ok(widths, npasses))
        return ORACLE_EINVAL;
    if (n > 0 && keys == NULL)
        return ORACLE_EINVAL;
    if (n < 2)
        return ORACLE_OK;
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 3
    /* planted mistake: the most significant pass is dropped */
    last = npasses - 1;
#endif
    ka = keys;
    kb = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (kb == NULL)
        return ORACLE_ENOMEM;
    if (vals != NULL) {
        va = vals;
        vb = (uint32_t *)malloc(n * sizeof(uint32_t));
        if (vb == NULL) {
            free(kb);
            return ORACLE_ENOMEM;
        }
    }
    for (p = 0; p < last; ++p) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 7
        /* planted mistake: digits taken most significant first */
        unsigned s = 32 - shift - widths[p];
#else
        unsigned s = shift;
#endif
        rc = oracle_counting_pass(ka, va, kb, vb, n, s, widths[p]);
        if (rc != ORACLE_OK)
            break;
        tmp = ka; ka = kb; kb = tmp;
        tmp = va; va = vb; vb = tmp;
        shift += widths[p];
    }
    /* the sorted data is in ka/va; bring it back into the caller's arrays */
    if (rc == ORACLE_OK && ka != keys) {
        memcpy(keys, ka, n * sizeof(uint32_t));
        if (vals != NULL)
            memcpy(vals, va, n * sizeof(uint32_t));
    }
    free(ka == keys ? kb : ka);
    if (vals != NULL)
        free(va == vals ? vb : va);
    return rc;
}

/*
 * Segmented form: segment s is [off[s], off[s+1]) and is sorted on its own
 * with the full LSD sort above; items outside [off[0], off[nseg]) are not
 * touched.  Offsets must be nondecreasing.
 */
int oracle_lsd_sort_segmented(uint32_t *keys, uint32_t *vals,
                              const uint32_t *off, uint32_t nseg,
                              const unsigned *widths, unsigned npasses)
{
    uint32_t s;
    int rc;
    if (!widths_ok(widths, npasses) || (off == NULL && nseg > 0))
        return ORACLE_EINVAL;
    for (s = 0; s < nseg; ++s)
        if (off[s + 1] < off[s])
            return ORACLE_EINVAL;
    for (s = 0; s < nseg; ++s) {
        uint64_t lo = off[s], len = (uint64_t)off[s + 1] - off[s];
        rc = oracle_lsd_sort(keys + lo, vals ? vals + lo : NULL, len, widths,
                             npasses);
        if (rc != ORACLE_OK)
            return rc;
    }
    return ORACLE_OK;
}

/*
 * "Reverse sorting" (Section 4, Algorithm 2) on one processing element,
 * with K = 32-bit keys and D = 8-bit digits numbered 0 (least significant)
 * to 3.  The buckets are growable arrays that items are appended to in the
 * order they are visited, as the paper's virtual-memory buckets are
 * (Section 3): no histogram is needed to fill them.  The steps, in the
 * algorithm's order:
 *
 *   1. each item is appended to buckets3[digit 3];
 *   2. bucketSizes = the sizes of buckets3, and outputIndices = its
 *      exclusive prefix sum: where each MSD bucket starts in the output;
 *   3. for every bucket3, in increasing MSD order:
 *        a. its items are appended to buckets0[digit 0];
 *        b. the items of buckets0, bucket by bucket in increasing digit
 *           order, are appended to buckets1[digit 1], and histogram2 counts
 *           their digit 2;
 *        c. the items of buckets1, bucket by bucket in increasing digit
 *           order, are written straight to the output: an item with digit 2
 *           equal to d goes to the bucket's start plus the number of the
 *           bucket's items with a smaller digit 2 plus the number of items
 *           with digit d already written.
 *
 * Reading of step 3c: the printed index adds outputIndices and histogram2
 * at the same digit d; that only makes sense with outputIndices taken at the
 * bucket's MSD and histogram2 turned into its exclusive prefix sum (counts
 * of smaller digits 2), which is what is written here.
 */
typedef struct {
    uint32_t *k, *v;
    uint64_t len, cap;
} obucket;

static int obucket_append(obucket *b, uint32_t k, uint32_t v, int with_v)
{
    if (b->len == b->cap) {
        uint64_t cap = b->cap ? 2 * b->cap : 16;
        uint32_t *nk = (uint32_t *)realloc(b->k, cap * sizeof(uint32_t));
        if (nk == NULL)
            return ORACLE_ENOMEM;
        b->k = nk;
        if (with_v) {
            uint32_t *nv = (uint32_t *)realloc(b->v, cap * sizeof(uint32_t));
            if (nv == NULL)
                return ORACLE_ENOMEM;
            b->v = nv;
        }
        b->cap = cap;
    }
    b->k[b->len] = k;
    if (with_v)
        b->v[b->len] = v;
    b->len += 1;
    return ORACLE_OK;
}

static void obuckets_free(obucket *b, unsigned count)
{
    unsigned i;
    for (i = 0; i < count; ++i) {
        free(b[i].k);
        free(b[i].v);
        b[i].k = b[i].v = NULL;
        b[i].len = b[i].cap = 0;
    }
}

#define OR_RADIX 256u

int oracle_reverse_sort(uint32_t *keys, uint32_t *vals, uint64_t n)
{
    obucket *buckets3, *buckets0, *buckets1;
    uint64_t bucket_sizes[OR_RADIX], output_indices[OR_RADIX];
    uint64_t histogram2[OR_RADIX], slot2[OR_RADIX];
    uint32_t *out_k = NULL, *out_v = NULL;
    uint64_t i, running;
    unsigned b3, b, d;
    const int with_v = vals != NULL;
    int rc = ORACLE_OK;
    if (n > 0 && keys == NULL)
        return ORACLE_EINVAL;
    if (n < 2)
        return ORACLE_OK;
    buckets3 = (obucket *)calloc(3 * OR_RADIX, sizeof(obucket));
    out_k = (uint32_t *)malloc(n * sizeof(uint32_t));
    out_v = with_v ? (uint32_t *)malloc(n * sizeof(uint32_t)) : NULL;
    if (buckets3 == NULL || out_k == NULL || (with_v && out_v == NULL)) {
        free(buckets3);
        free(out_k);
        free(out_v);
        return ORACLE_ENOMEM;
    }
    buckets0 = buckets3 + OR_RADIX;
    buckets1 = buckets0 + OR_RADIX;

    /* 1: partition by the most significant digit */
    for (i = 0; i < n && rc == ORACLE_OK; ++i) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 9
        /* planted mistake: the partition takes digit 2 for the MSD */
        const uint32_t d3 = digit_of(keys[i], 16, 8);
#else
        const uint32_t d3 = digit_of(keys[i], 24, 8);
#endif
        rc = obucket_append(&buckets3[d3], keys[i], with_v ? vals[i] : 0u, with_v);
    }

    /* 2: bucket sizes and where each MSD bucket starts in the output */
    running = 0;
    for (d = 0; d < OR_RADIX; ++d) {
        bucket_sizes[d] = buckets3[d].len;
        output_indices[d] = running;
        running += bucket_sizes[d];
    }

    /* 3: local LSD passes over digits 0, 1, 2 of each MSD bucket */
    for (b3 = 0; b3 < OR_RADIX && rc == ORACLE_OK; ++b3) {
        const obucket *src = &buckets3[b3];
        /* 3a */
        for (i = 0; i < src->len && rc == ORACLE_OK; ++i)
            rc = obucket_append(&buckets0[digit_of(src->k[i], 0, 8)], src->k[i],
                                with_v ? src->v[i] : 0u, with_v);
        /* 3b */
        for (d = 0; d < OR_RADIX; ++d)
            histogram2[d] = 0;
        for (b = 0; b < OR_RADIX && rc == ORACLE_OK; ++b) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 10
            /* planted mistake: buckets0 visited in decreasing digit order */
            const obucket *b0 = &buckets0[OR_RADIX - 1 - b];
#else
            const obucket *b0 = &buckets0[b];
#endif
            for (i = 0; i < b0->len && rc == ORACLE_OK; ++i) {
                rc = obucket_append(&buckets1[digit_of(b0->k[i], 8, 8)], b0->k[i],
                                    with_v ? b0->v[i] : 0u, with_v);
                histogram2[digit_of(b0->k[i], 16, 8)] += 1;
            }
        }
        /* 3c */
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 8
        /* planted mistake: every bucket is written from output slot 0 */
        running = 0 * output_indices[b3];
#else
        running = output_indices[b3];
#endif
        for (d = 0; d < OR_RADIX; ++d) {
            slot2[d] = running;
            running += histogram2[d];
        }
        for (b = 0; b < OR_RADIX && rc == ORACLE_OK; ++b) {
            const obucket *b1 = &buckets1[b];
            for (i = 0; i < b1->len; ++i) {
                uint32_t dd = digit_of(b1->k[i], 16, 8);
                out_k[slot2[dd]] = b1->k[i];
                if (with_v)
                    out_v[slot2[dd]] = b1->v[i];
                slot2[dd] += 1;
            }
        }
        obuckets_free(buckets0, OR_RADIX);
        obuckets_free(buckets1, OR_RADIX);
    }
    if (rc == ORACLE_OK) {
        memcpy(keys, out_k, n * sizeof(uint32_t));
        if (with_v)
            memcpy(vals, out_v, n * sizeof(uint32_t));
    }
    obuckets_free(buckets3, 3 * OR_RADIX);
    free(buckets3);
    free(out_k);
    free(out_v);
    return rc;
}

/*
 * 64-bit keys (the wider items Section 4 allows: a key with a value
 * adjacent to it, larger combinations than one 64-bit word being possible).
 * The same LSD radix sort as above, on K = 64-bit keys: digit widths sum to
 * 64, each pass is Section 3's counting sort on one digit, and each item's
 * value of vw 32-bit words (0, 1 or 2) moves with its key.
 */
static uint32_t digit_of64(uint64_t key, unsigned shift, unsigned width)
{
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 11
    /* planted mistake: the shift wraps at 32 bits */
    return (uint32_t)(key >> (shift & 31u)) & ((1u << width) - 1u);
#else
    return (uint32_t)(key >> shift) & ((1u << width) - 1u);
#endif
}

static int oracle_counting_pass64(const uint64_t *kin, const uint32_t *vin,
                                  uint64_t *kout, uint32_t *vout, unsigned vw,
                                  uint64_t n, unsigned shift, unsigned width)
{
    uint64_t buckets = (uint64_t)1 << width, d, i, running = 0;
    uint64_t *next = (uint64_t *)calloc(buckets, sizeof(uint64_t));
    unsigned w;
    if (next == NULL)
        return ORACLE_ENOMEM;
    for (i = 0; i < n; ++i) /* histogram */
        next[digit_of64(kin[i], shift, width)] += 1;
    for (d = 0; d < buckets; ++d) { /* exclusive prefix sum */
        uint64_t count = next[d];
        next[d] = running;
        running += count;
    }
    for (i = 0; i < n; ++i) { /* scatter in input order */
        uint32_t dd = digit_of64(kin[i], shift, width);
        uint64_t slot = next[dd];
        kout[slot] = kin[i];
        for (w = 0; w < vw; ++w) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 12
            /* planted mistake: only the first value word moves */
            vout[slot * vw + w] = w == 0 ? vin[i * vw] : vin[slot * vw + w];
#else
            vout[slot * vw + w] = vin[i * vw + w];
#endif
        }
        next[dd] = slot + 1;
    }
    free(next);
    return ORACLE_OK;
}

int oracle_lsd_sort64(uint64_t *keys, uint32_t *vals, unsigned vw, uint64_t n,
                      const unsigned *widths, unsigned npasses)
{
    uint64_t *ka, *kb, *tk;
    uint32_t *va = NULL, *vb = NULL, *tv;
    unsigned p, shift = 0, total = 0;
    int rc = ORACLE_OK;
    if (widths == NULL || npasses == 0 || npasses > 64 || vw > 2 || (vw > 0 && vals == NULL))
        return ORACLE_EINVAL;
    for (p = 0; p < npasses; ++p) {
        if (widths[p] < 1 || widths[p] > 16)
            return ORACLE_EINVAL;
        total += widths[p];
    }
    if (total != 64 || (n > 0 && keys == NULL))
        return ORACLE_EINVAL;
    if (n < 2)
        return ORACLE_OK;
    ka = keys;
    kb = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (kb == NULL)
        return ORACLE_ENOMEM;
    if (vw > 0) {
        va = vals;
        vb = (uint32_t *)malloc(n * vw * sizeof(uint32_t));
        if (vb == NULL) {
            free(kb);
            return ORACLE_ENOMEM;
        }
    }
    for (p = 0; p < npasses && rc == ORACLE_OK; ++p) {
        rc = oracle_counting_pass64(ka, va, kb, vb, vw, n, shift, widths[p]);
        tk = ka; ka = kb; kb = tk;
        tv = va; va = vb; vb = tv;
        shift += widths[p];
    }
    if (rc == ORACLE_OK && ka != keys) {
        memcpy(keys, ka, n * sizeof(uint64_t));
        if (vw > 0)
            memcpy(vals, va, n * vw * sizeof(uint32_t));
    }
    free(ka == keys ? kb : ka);
    if (vw > 0)
        free(va == vals ? vb : va);
    return rc;
}
