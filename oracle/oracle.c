/*
 * CPU oracle for the Diverting Fast Radix (DFR) sort, arXiv 2207.14334.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  The GPU product path never calls, links or
 * includes anything in this directory, and this file includes nothing from it.
 *
 * What the method computes.  DFR deals the top digits least-significant first,
 * which is stable (Sec. 2.1), diverts runs of small buckets to a simple stable
 * sort (Sec. 3, diversion paragraph; stability of insertion and merge sort, Sec. 2.2)
 * and recurses on large buckets, whose records already share their leading
 * digits (Sec. 2.2, MSD paragraph).  Its result is therefore the plain stable sort
 * of the records by key, which has a closed definition:
 *
 *     record i lands at  rank(i) = #{ j : k_j < k_i } + #{ j < i : k_j == k_i }
 *
 * with keys compared as unsigned integers.  oracle_stable_sort writes that
 * definition out (sort by the pair (key, original index)); oracle_rank evaluates the
 * formula directly in O(n^2) for tiny inputs.
 *
 * The stage functions follow the paper's vocabulary (Sec. 2): a *count* builds the
 * occurrence counts of one digit, the counts become indices by an exclusive prefix
 * sum, and a *deal* places every record at index[digit]++ .  oracle_lsd_sort chains
 * deals from the least significant digit (Sec. 2.1), and oracle_dfr_sort takes the
 * DFR steps in the order the prose of Sec. 3 gives them (estimate the number of top
 * digits, LSD-sort those, divert runs of small buckets to insertion sort, recurse
 * on large buckets).  Those three produce the same result as the definition; the
 * tests pin them to it and to outside references (brute force, numpy).
 *
 * Conventions: keys are 4 or 8 bytes (kb), payloads 0, 4 or 8 bytes (vb, 0 = none),
 * arrays are contiguous, little-endian, structure-of-arrays.  Functions return 0 on
 * success, -1 on a bad argument, -2 when host memory runs out.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EARG (-1)
#define OR_ENOMEM (-2)

static uint64_t ld(const void* p, int w, size_t i) {
    return w == 4 ? (uint64_t)((const uint32_t*)p)[i] : ((const uint64_t*)p)[i];
}

static void st(void* p, int w, size_t i, uint64_t v) {
    if (w == 4)
        ((uint32_t*)p)[i] = (uint32_t)v;
    else
        ((uint64_t*)p)[i] = v;
}

static int widths_ok(int kb, int vb) {
    return (kb == 4 || kb == 8) && (vb == 0 || vb == 4 || vb == 8);
}

/* ------------------------------------------------------------------------------ */
/* The definition: sort by (key, original index).                                  */
/* ------------------------------------------------------------------------------ */

typedef struct {
    uint64_t key;
    uint64_t idx;
} keyed_index;

static int cmp_key_then_index(const void* a, const void* b) {
    const keyed_index* x = (const keyed_index*)a;
    const keyed_index* y = (const keyed_index*)b;
#ifdef ORACLE_PLANT_SIGNED_COMPARE
    /* Planted mistake for the pin tests: compare keys as signed integers. */
    int64_t xs = x->key, ys = y->key;
    if (x->key <= 0xffffffffu && y->key <= 0xffffffffu) {
        xs = (int32_t)(uint32_t)x->key;
        ys = (int32_t)(uint32_t)y->key;
    }
    if (xs != ys) return xs < ys ? -1 : 1;
#else
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
#endif
#ifdef ORACLE_PLANT_REVERSED_TIES
    /* Planted mistake for the pin tests: equal keys leave in reverse input order. */
    return (x->idx < y->idx) - (x->idx > y->idx);
#else
    return (x->idx > y->idx) - (x->idx < y->idx);
#endif
}

/* Stable sort of n records (Sec. 2.1 stability; Sec. 3 DFR result).  out_* may not
 * alias the inputs.  vals / out_vals are ignored when vb == 0. */
int oracle_stable_sort(const void* keys, const void* vals, size_t n, int kb, int vb,
                       void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb)) return OR_EARG;
    if (n == 0) return OR_OK;
    if (!keys || !out_keys || (vb && (!vals || !out_vals))) return OR_EARG;
    keyed_index* r = (keyed_index*)malloc(n * sizeof(keyed_index));
    if (!r) return OR_ENOMEM;
    for (size_t i = 0; i < n; ++i) {
        r[i].key = ld(keys, kb, i);
        r[i].idx = i;
    }
    qsort(r, n, sizeof(keyed_index), cmp_key_then_index);
#ifdef ORACLE_PLANT_DROP_LAST
    /* Planted mistake for the pin tests: the last record is replaced by the first. */
    if (n > 1) r[n - 1] = r[0];
#endif
    for (size_t i = 0; i < n; ++i) {
        st(out_keys, kb, i, r[i].key);
        if (vb) st(out_vals, vb, i, ld(vals, vb, r[i].idx));
    }
    free(r);
    return OR_OK;
}

/* ------------------------------------------------------------------------------ */
/* The same definition on several host threads, for timing the CPU baseline: each    */
/* thread sorts one contiguous chunk of the records by (key, index) as above, then    */
/* neighbouring sorted runs are merged pairwise, level by level, into one run.  A     */
/* merge that takes the left run's record while its key is not greater than the       */
/* right run's keeps equal keys in input order (every left record precedes every      */
/* right one in the input), so the result is the same stable sort.                    */
/* ------------------------------------------------------------------------------ */

typedef struct {
    keyed_index* r;
    size_t lo, hi;
} sort_job;

static void* sort_chunk(void* arg) {
    sort_job* j = (sort_job*)arg;
    qsort(j->r + j->lo, j->hi - j->lo, sizeof(keyed_index), cmp_key_then_index);
    return NULL;
}

typedef struct {
    const keyed_index* src;
    keyed_index* dst;
    size_t lo, mid, hi;  /* merges src[lo, mid) and src[mid, hi) into dst[lo, hi) */
} merge_job;

static void* merge_runs(void* arg) {
    merge_job* m = (merge_job*)arg;
    size_t a = m->lo, b = m->mid, o = m->lo;
    while (a < m->mid && b < m->hi) {
#ifdef ORACLE_PLANT_MERGE_RIGHT_FIRST
        /* Planted mistake for the pin tests: equal keys take the right run first. */
        if (m->src[a].key < m->src[b].key)
#else
        if (m->src[a].key <= m->src[b].key)
#endif
            m->dst[o++] = m->src[a++];
        else
            m->dst[o++] = m->src[b++];
    }
    while (a < m->mid) m->dst[o++] = m->src[a++];
    while (b < m->hi) m->dst[o++] = m->src[b++];
    return NULL;
}

int oracle_stable_sort_parallel(const void* keys, const void* vals, size_t n, int kb, int vb,
                                int threads, void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb) || threads < 1) return OR_EARG;
    if (n == 0) return OR_OK;
    if (!keys || !out_keys || (vb && (!vals || !out_vals))) return OR_EARG;
    size_t p = (size_t)threads < n ? (size_t)threads : n;
    keyed_index* r = (keyed_index*)malloc(n * sizeof(keyed_index));
    keyed_index* t = (keyed_index*)malloc(n * sizeof(keyed_index));
    size_t* bound = (size_t*)malloc((p + 1) * sizeof(size_t));
    pthread_t* th = (pthread_t*)malloc(p * sizeof(pthread_t));
    sort_job* sj = (sort_job*)malloc(p * sizeof(sort_job));
    merge_job* mj = (merge_job*)malloc(p * sizeof(merge_job));
    if (!r || !t || !bound || !th || !sj || !mj) {
        free(r); free(t); free(bound); free(th); free(sj); free(mj);
        return OR_ENOMEM;
    }
    for (size_t i = 0; i < n; ++i) {
        r[i].key = ld(keys, kb, i);
        r[i].idx = i;
    }
    for (size_t c = 0; c <= p; ++c) bound[c] = n / p * c + (c < n % p ? c : n % p);
    for (size_t c = 0; c < p; ++c) {
        sj[c].r = r;
        sj[c].lo = bound[c];
        sj[c].hi = bound[c + 1];
        if (pthread_create(&th[c], NULL, sort_chunk, &sj[c]) != 0) sort_chunk(&sj[c]), th[c] = 0;
    }
    for (size_t c = 0; c < p; ++c)
        if (th[c]) pthread_join(th[c], NULL);
    /* Runs are [bound[c], bound[c + 1]); each level merges runs 2i and 2i + 1. */
    size_t runs = p;
    keyed_index *src = r, *dst = t;
    while (runs > 1) {
        size_t m = 0;
        for (size_t c = 0; c < runs; c += 2) {
            mj[m].src = src;
            mj[m].dst = dst;
            mj[m].lo = bound[c];
            mj[m].mid = bound[c + 1];  /* a last unpaired run is copied as it is */
            mj[m].hi = c + 1 < runs ? bound[c + 2] : bound[c + 1];
            if (pthread_create(&th[m], NULL, merge_runs, &mj[m]) != 0) merge_runs(&mj[m]), th[m] = 0;
            ++m;
        }
        for (size_t c = 0; c < m; ++c)
            if (th[c]) pthread_join(th[c], NULL);
        for (size_t c = 0; c < m; ++c) bound[c] = mj[c].lo;
        bound[m] = n;
        runs = m;
        keyed_index* x = src;
        src = dst;
        dst = x;
    }
    for (size_t i = 0; i < n; ++i) {
        st(out_keys, kb, i, src[i].key);
        if (vb) st(out_vals, vb, i, ld(vals, vb, src[i].idx));
    }
    free(r); free(t); free(bound); free(th); free(sj); free(mj);
    return OR_OK;
}

/* ------------------------------------------------------------------------------ */
/* Signed and floating-point keys (beyond the paper, which sorts unsigned integers). */
/* The order is written out from its definition, comparing the decoded values:     */
/* two's-complement integers by value; binary floats by IEEE 754 totalOrder:       */
/* negative before positive (by the sign bit, so -0 < +0 and -NaN < +NaN), and      */
/* within one sign by magnitude (the exponent-and-fraction field read as an        */
/* unsigned integer, which orders zero < subnormals < normals < infinity < NaNs by  */
/* payload), the larger magnitude first for negatives.                             */
/* ------------------------------------------------------------------------------ */

#define ORACLE_KEY_U32 0
#define ORACLE_KEY_U64 1
#define ORACLE_KEY_I32 2
#define ORACLE_KEY_I64 3
#define ORACLE_KEY_F32 4
#define ORACLE_KEY_F64 5

static int ties(const keyed_index* x, const keyed_index* y) {
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int cmp_i32(const void* a, const void* b) {
    const keyed_index *x = (const keyed_index*)a, *y = (const keyed_index*)b;
    const int32_t u = (int32_t)(uint32_t)x->key, v = (int32_t)(uint32_t)y->key;
    if (u != v) return u < v ? -1 : 1;
    return ties(x, y);
}

static int cmp_i64(const void* a, const void* b) {
    const keyed_index *x = (const keyed_index*)a, *y = (const keyed_index*)b;
    const int64_t u = (int64_t)x->key, v = (int64_t)y->key;
    if (u != v) return u < v ? -1 : 1;
    return ties(x, y);
}

/* totalOrder of two encodings of `bits` bits: sign, then magnitude. */
static int total_order(uint64_t x, uint64_t y, int bits) {
    const uint64_t sign = 1ull << (bits - 1), mag = sign - 1;
    const int xn = (x & sign) != 0, yn = (y & sign) != 0;
    if (xn != yn) return xn ? -1 : 1;
    const uint64_t mx = x & mag, my = y & mag;
    if (mx == my) return 0;
#ifdef ORACLE_PLANT_FLOAT_NO_REVERSE
    /* Planted mistake for the pin tests: negatives ordered by increasing magnitude. */
    return mx < my ? -1 : 1;
#else
    if (xn) return mx > my ? -1 : 1;  /* both negative: larger magnitude is smaller */
    return mx < my ? -1 : 1;
#endif
}

static int cmp_f32(const void* a, const void* b) {
    const keyed_index *x = (const keyed_index*)a, *y = (const keyed_index*)b;
    const int c = total_order(x->key, y->key, 32);
    return c ? c : ties(x, y);
}

static int cmp_f64(const void* a, const void* b) {
    const keyed_index *x = (const keyed_index*)a, *y = (const keyed_index*)b;
    const int c = total_order(x->key, y->key, 64);
    return c ? c : ties(x, y);
}

/* Stable sort under the order of key_type (ORACLE_KEY_*); keys hold the raw encodings
 * (4 bytes for the 32-bit types, 8 for the 64-bit ones). */
int oracle_stable_sort_typed(const void* keys, const void* vals, size_t n, int key_type, int vb,
                             void* out_keys, void* out_vals) {
    if (key_type < ORACLE_KEY_U32 || key_type > ORACLE_KEY_F64) return OR_EARG;
    const int kb = (key_type % 2 == 0) ? 4 : 8;
    if (!widths_ok(kb, vb)) return OR_EARG;
    if (key_type <= ORACLE_KEY_U64) return oracle_stable_sort(keys, vals, n, kb, vb, out_keys, out_vals);
    if (n == 0) return OR_OK;
    if (!keys || !out_keys || (vb && (!vals || !out_vals))) return OR_EARG;
    keyed_index* r = (keyed_index*)malloc(n * sizeof(keyed_index));
    if (!r) return OR_ENOMEM;
    for (size_t i = 0; i < n; ++i) {
        r[i].key = ld(keys, kb, i);
        r[i].idx = i;
    }
    int (*cmp)(const void*, const void*) = key_type == ORACLE_KEY_I32   ? cmp_i32
                                           : key_type == ORACLE_KEY_I64 ? cmp_i64
                                           : key_type == ORACLE_KEY_F32 ? cmp_f32
                                                                        : cmp_f64;
    qsort(r, n, sizeof(keyed_index), cmp);
    for (size_t i = 0; i < n; ++i) {
        st(out_keys, kb, i, r[i].key);
        if (vb) st(out_vals, vb, i, ld(vals, vb, r[i].idx));
    }
    free(r);
    return OR_OK;
}

/* Segmented form: every segment [off[s], off[s+1]) is sorted on its own.
 * off has S+1 entries, off[0] == 0, non-decreasing, off[S] == n. */
int oracle_segmented_sort(const void* keys, const void* vals, size_t n, int kb, int vb,
                          const uint64_t* off, size_t S, void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb) || !off) return OR_EARG;
    if (off[0] != 0 || off[S] != n) return OR_EARG;
    for (size_t s = 0; s < S; ++s)
        if (off[s + 1] < off[s]) return OR_EARG;
    for (size_t s = 0; s < S; ++s) {
        size_t a = off[s], len = off[s + 1] - off[s];
        if (len == 0) continue;
        const char* kin = (const char*)keys + a * kb;
        char* kout = (char*)out_keys + a * kb;
        const char* vin = vb ? (const char*)vals + a * vb : NULL;
        char* vout = vb ? (char*)out_vals + a * vb : NULL;
        int rc = oracle_stable_sort(kin, vin, len, kb, vb, kout, vout);
        if (rc) return rc;
    }
    return OR_OK;
}

/* The rank formula itself, O(n^2): rank[i] = #{j: k_j < k_i} + #{j < i: k_j == k_i}. */
int oracle_rank(const void* keys, size_t n, int kb, uint64_t* rank) {
    if (!(kb == 4 || kb == 8)) return OR_EARG;
    for (size_t i = 0; i < n; ++i) {
        uint64_t ki = ld(keys, kb, i), r = 0;
        for (size_t j = 0; j < n; ++j) {
            uint64_t kj = ld(keys, kb, j);
            if (kj < ki || (kj == ki && j < i)) ++r;
        }
        rank[i] = r;
    }
    return OR_OK;
}

/* rank(i) of one record in O(n), for sampling outputs of very large sorts. */
uint64_t oracle_rank_of(const void* keys, size_t n, int kb, size_t i) {
    uint64_t ki = ld(keys, kb, i), r = 0;
    for (size_t j = 0; j < n; ++j) {
        uint64_t kj = ld(keys, kb, j);
        r += (kj < ki) | ((kj == ki) & (j < i));
    }
    return r;
}

/* ------------------------------------------------------------------------------ */
/* Count and deal (Sec. 2, counting sort paragraph and its count[10] example).      */
/* ------------------------------------------------------------------------------ */

static uint64_t digit_of(uint64_t key, int shift, int bits) {
    return (key >> shift) & ((1ull << bits) - 1);
}

static int digit_args_ok(int kb, int shift, int bits) {
    return bits >= 1 && bits <= 16 && shift >= 0 && shift + bits <= 8 * kb;
}

/* count: hist[v] = number of records whose digit (key >> shift) mod 2^bits equals v. */
int oracle_count(const void* keys, size_t n, int kb, int shift, int bits, uint64_t* hist) {
    if (!(kb == 4 || kb == 8) || !digit_args_ok(kb, shift, bits) || !hist) return OR_EARG;
    memset(hist, 0, sizeof(uint64_t) << bits);
    for (size_t i = 0; i < n; ++i) hist[digit_of(ld(keys, kb, i), shift, bits)]++;
    return OR_OK;
}

/* One counting-sort pass on one digit: count, turn the counts into indices by an
 * exclusive prefix sum, then deal each record to buff[index[digit]++]. */
int oracle_deal(const void* keys, const void* vals, size_t n, int kb, int vb, int shift,
                int bits, void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb) || !digit_args_ok(kb, shift, bits)) return OR_EARG;
    if (n == 0) return OR_OK;
    size_t M = (size_t)1 << bits;
    uint64_t* index = (uint64_t*)malloc(M * sizeof(uint64_t));
    if (!index) return OR_ENOMEM;
    oracle_count(keys, n, kb, shift, bits, index);
    uint64_t run = 0;
    for (size_t v = 0; v < M; ++v) {
        uint64_t c = index[v];
        index[v] = run;
#ifdef ORACLE_PLANT_INCLUSIVE_SCAN
        /* Planted mistake for the pin tests: inclusive instead of exclusive sum. */
        index[v] = run + c - (c ? 1 : 0);
#endif
        run += c;
    }
    for (size_t i = 0; i < n; ++i) {
        uint64_t k = ld(keys, kb, i);
        uint64_t dst = index[digit_of(k, shift, bits)]++;
        if (dst >= n) { free(index); return OR_EARG; }
        st(out_keys, kb, dst, k);
        if (vb) st(out_vals, vb, dst, ld(vals, vb, i));
    }
    free(index);
    return OR_OK;
}

/* LSD radix sort (Sec. 2.1): deal on every digit from least to most significant,
 * alternating between the input copy and a buffer; the last deal lands in out. */
int oracle_lsd_sort(const void* keys, const void* vals, size_t n, int kb, int vb, int bits,
                    void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb) || bits < 1 || bits > 16) return OR_EARG;
    if (n == 0) return OR_OK;
    int ndig = (8 * kb + bits - 1) / bits;
    void* ka = malloc(n * kb);
    void* kbuf = malloc(n * kb);
    void* va = vb ? malloc(n * vb) : NULL;
    void* vbuf = vb ? malloc(n * vb) : NULL;
    if (!ka || !kbuf || (vb && (!va || !vbuf))) {
        free(ka); free(kbuf); free(va); free(vbuf);
        return OR_ENOMEM;
    }
    memcpy(ka, keys, n * kb);
    if (vb) memcpy(va, vals, n * vb);
    int rc = OR_OK;
    for (int j = 0; j < ndig && rc == OR_OK; ++j) {
        int shift = j * bits;
        int w = shift + bits <= 8 * kb ? bits : 8 * kb - shift;
        rc = oracle_deal(ka, va, n, kb, vb, shift, w, kbuf, vbuf);
        void* t = ka; ka = kbuf; kbuf = t;
        t = va; va = vbuf; vbuf = t;
    }
    if (rc == OR_OK) {
        memcpy(out_keys, ka, n * kb);
        if (vb) memcpy(out_vals, va, n * vb);
    }
    free(ka); free(kbuf); free(va); free(vbuf);
    return rc;
}

/* Bucket starts after the leading digits have been dealt: the positions p where
 * p == 0 or (key[p] >> lo_bit) != (key[p-1] >> lo_bit).  Returns how many there are;
 * writes at most cap of them. */
size_t oracle_bucket_starts(const void* keys, size_t n, int kb, int lo_bit, uint64_t* starts,
                            size_t cap) {
    size_t c = 0;
    for (size_t p = 0; p < n; ++p) {
        int head = p == 0;
        if (!head) {
            uint64_t a = ld(keys, kb, p - 1), b = ld(keys, kb, p);
            head = lo_bit >= 64 ? 0 : (a >> lo_bit) != (b >> lo_bit);
        }
        if (head) {
            if (c < cap && starts) starts[c] = p;
            ++c;
        }
    }
    return c;
}

/* ------------------------------------------------------------------------------ */
/* DFR, step by step (Sec. 3, diverting LSD paragraph and the analysis of Sec. 3.1).  */
/* ------------------------------------------------------------------------------ */

/* Stable insertion sort of a run of records by full key (the diversion of Sec. 2.2
 * and Sec. 3).  The run is already ordered by its buckets' prefixes, so records only
 * move inside their own bucket. */
static void insertion_sort_run(void* k, void* v, int kb, int vb, size_t a, size_t b) {
    for (size_t i = a + 1; i < b; ++i) {
        uint64_t key = ld(k, kb, i), val = vb ? ld(v, vb, i) : 0;
        size_t j = i;
        while (j > a && ld(k, kb, j - 1) > key) {
            st(k, kb, j, ld(k, kb, j - 1));
            if (vb) st(v, vb, j, ld(v, vb, j - 1));
            --j;
        }
        st(k, kb, j, key);
        if (vb) st(v, vb, j, val);
    }
}

/* Number of top digits to deal so that, for keys spread uniformly over the digits
 * that remain, the expected bucket holds at most `divert` records: the smallest d
 * with n / M^d <= divert, capped at the digits left (Sec. 3; Sec. 3.1 on N_d). */
static int estimate_top_digits(size_t n, int bits, int digits_left, size_t divert) {
    int d = 0;
    double expect = (double)n;
    while (d < digits_left && expect > (double)divert) {
        expect /= (double)(1ull << bits);
        ++d;
    }
    return d;
}

/* Sorts the records k[a..b) / v[a..b) in place, whose keys agree on all bits at and
 * above `hi_bit`; digits of `bits` bits are taken downward from hi_bit. */
static int dfr_rec(void* k, void* v, void* kt, void* vt, int kb, int vb, int bits, size_t divert,
                   size_t a, size_t b, int hi_bit) {
    size_t n = b - a;
    if (n <= 1 || hi_bit <= 0) return OR_OK; /* no digits left: all keys equal */
    if (n <= divert) {
        insertion_sort_run(k, v, kb, vb, a, b);
        return OR_OK;
    }
    int digits_left = (hi_bit + bits - 1) / bits;
    int d = estimate_top_digits(n, bits, digits_left, divert);
    if (d < 1) d = 1;
    /* LSD over the top d digits: least significant of them first. */
    int lo_bit = hi_bit - d * bits;
    if (lo_bit < 0) lo_bit = 0;
    char* K = (char*)k + a * kb;
    char* V = vb ? (char*)v + a * vb : NULL;
    char* KT = (char*)kt + a * kb;
    char* VT = vb ? (char*)vt + a * vb : NULL;
    for (int shift = lo_bit; shift < hi_bit; shift += bits) {
        int w = shift + bits <= hi_bit ? bits : hi_bit - shift;
        int rc = oracle_deal(K, V, n, kb, vb, shift, w, KT, VT);
        if (rc) return rc;
        memcpy(K, KT, n * kb);
        if (vb) memcpy(V, VT, n * vb);
    }
    /* Walk the buckets of equal prefix (key >> lo_bit): runs of small buckets are
     * insertion-sorted as one unit, large buckets recurse on the remaining digits. */
    size_t p = a, run_start = a;
    while (p < b) {
        size_t q = p + 1;
        uint64_t pre = lo_bit >= 64 ? 0 : ld(k, kb, p) >> lo_bit;
        while (q < b && (lo_bit >= 64 ? 0 : ld(k, kb, q) >> lo_bit) == pre) ++q;
        if (q - p > divert) {
            insertion_sort_run(k, v, kb, vb, run_start, p);
            int rc = dfr_rec(k, v, kt, vt, kb, vb, bits, divert, p, q, lo_bit);
            if (rc) return rc;
            run_start = q;
        }
        p = q;
    }
    insertion_sort_run(k, v, kb, vb, run_start, b);
    return OR_OK;
}

/* DFR following the paper's steps; `divert` is the diversion threshold N_d. */
int oracle_dfr_sort(const void* keys, const void* vals, size_t n, int kb, int vb, int bits,
                    size_t divert, void* out_keys, void* out_vals) {
    if (!widths_ok(kb, vb) || bits < 1 || bits > 16 || divert < 1) return OR_EARG;
    if (n == 0) return OR_OK;
    void* kt = malloc(n * kb);
    void* vt = vb ? malloc(n * vb) : NULL;
    if (!kt || (vb && !vt)) { free(kt); free(vt); return OR_ENOMEM; }
    memcpy(out_keys, keys, n * kb);
    if (vb) memcpy(out_vals, vals, n * vb);
    int rc = dfr_rec(out_keys, out_vals, kt, vt, kb, vb, bits, divert, 0, n, 8 * kb);
    free(kt); free(vt);
    return rc;
}

/* ------------------------------------------------------------------------------ */
/* Property checker for outputs too large to sort on the host at test time.        */
/* ------------------------------------------------------------------------------ */

/* With the index payload v_i = i the stable sort is the only output for which
 *   (1) out_vals is a permutation of 0..n-1,
 *   (2) out_keys[p] == in_keys[out_vals[p]],
 *   (3) out_keys is non-decreasing, and
 *   (4) equal neighbouring keys carry increasing out_vals.
 * Returns -1 when all hold, else the first position p that breaks one, and the
 * broken property's number in *what. */
int64_t oracle_check_index_payload(const void* in_keys, size_t n, int kb, const void* out_keys,
                                   const void* out_vals, int vb, int* what) {
    *what = 0;
    uint8_t* seen = (uint8_t*)calloc(n ? n : 1, 1);
    if (!seen) { *what = -2; return 0; }
    for (size_t p = 0; p < n; ++p) {
        uint64_t src = ld(out_vals, vb, p);
        if (src >= n || seen[src]) { *what = 1; free(seen); return (int64_t)p; }
        seen[src] = 1;
        uint64_t k = ld(out_keys, kb, p);
        if (k != ld(in_keys, kb, src)) { *what = 2; free(seen); return (int64_t)p; }
        if (p > 0) {
            uint64_t kp = ld(out_keys, kb, p - 1);
            if (kp > k) { *what = 3; free(seen); return (int64_t)p; }
            if (kp == k && ld(out_vals, vb, p - 1) >= src) { *what = 4; free(seen); return (int64_t)p; }
        }
    }
    free(seen);
    return -1;
}

/* ------------------------------------------------------------------------------ */
/* Fast Radix's estimated buckets (Sec. 3.1, Eq. 2).  N uniform records dealt into M */
/* buckets of N/M slots each: a bucket that receives k < N/M records leaves          */
/* N/M - k slots empty, and as many records overflow elsewhere.  The expected        */
/* overflow as a fraction of N is the sum over k < ceil(N/M) of Eq. 2's term          */
/*     (N/M - k) (M/N) C(N, k) (1/M)^k (1 - 1/M)^(N-k),                              */
/* the binomial probability of k records in one bucket times its empty slots, over   */
/* the M buckets.  Terms are evaluated in log space (lgamma) so that N may be large. */
/* ------------------------------------------------------------------------------ */
double oracle_overflow_fraction(uint64_t N, uint32_t M) {
    if (N == 0 || M < 2) return 0.0;
    const double n = (double)N, m = (double)M, cap = n / m;
#ifdef ORACLE_PLANT_OVERFLOW_EXTRA_TERM
    /* Planted mistake for the pin tests: one term too many. */
    const uint64_t kmax = (N + M - 1) / M + 1;
#else
    const uint64_t kmax = (N + M - 1) / M;  /* ceil(N/M): k runs over [0, kmax) */
#endif
    const double lp = log(1.0 / m), lq = log1p(-1.0 / m), lgn = lgamma(n + 1.0);
    double sum = 0.0;
    for (uint64_t k = 0; k < kmax; ++k) {
        const double kk = (double)k;
        const double lbin = lgn - lgamma(kk + 1.0) - lgamma(n - kk + 1.0) + kk * lp + (n - kk) * lq;
        sum += (cap - kk) * (m / n) * exp(lbin);
    }
    return sum;
}
