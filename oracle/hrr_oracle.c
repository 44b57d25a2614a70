/*
 * hrr_oracle.c -- CPU oracle for hierarchical Russian-roulette culling with a
 * Cranley-Patterson rotated base-2 radical inverse (Pantaleoni,
 * "Blue-Noise Dithered QMC Hierarchical Russian Roulette").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * Everything here is written as the plain definition of what the hot path
 * computes, slow on purpose:
 *   - the radical inverse reverses digits one bit at a time (Section 2, the
 *     definition of Phi_b);
 *   - the range minimum scans every index of [a,b) (Section 1, the equations
 *     for v(a,b) and for its argmin k);
 *   - the culled pair set is the all-pairs leaf test, no hierarchy at all:
 *     hierarchical Russian roulette must return exactly the pairs whose own
 *     random number passes its own acceptance test (Section 1, the HRR
 *     setting);
 *   - the dyadic closed form is a second, independent way to get the range
 *     minimum of very long ranges that a scan cannot reach.  It is pinned to
 *     the scan by the tests before it is trusted.
 *
 * Fixed-point convention: a value in [0,1) with B bits is stored as the
 * integer floor(x * 2^B), so Phi_2(i) = bitrev_B(i) / 2^B exactly and
 * (Phi_2(i) + r) mod 1 = ((bitrev_B(i) + R) mod 2^B) / 2^B with R = r * 2^B.
 *
 * Floating point: the acceptance test is evaluated in IEEE binary32 with every
 * operation rounded separately (build with -ffp-contract=off, SSE math, no
 * fast-math), because a float decides an integer there and both sides must
 * take that decision in the same precision.
 *
 * Build:  python oracle/build.py   (gcc -O2 -ffp-contract=off -shared -fPIC)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Radical inverse and the shifted sequence (Section 1 and Section 2).        */
/* ------------------------------------------------------------------------- */

/* Phi_2 in B-bit fixed point: the binary digits of i, reversed.  Digit k of
 * i (weight 2^k) becomes weight 2^(B-1-k), i.e. 2^-(k+1) after the point. */
OR_EXPORT uint64_t or_bitrev(uint64_t i, int B) {
    uint64_t y = 0;
    for (int k = 0; k < B; ++k)
        if ((i >> k) & 1u) y |= (uint64_t)1 << (B - 1 - k);
    return y;
}

static uint64_t mask_bits(int B) { return B >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << B) - 1); }

/* phi(i) = (Phi_2(i) + r) mod 1, B-bit fixed point. */
OR_EXPORT uint64_t or_phi(uint64_t i, uint64_t r, int B) {
    return (or_bitrev(i, B) + r) & mask_bits(B);
}

/* v(a,b) and its argmin by scanning every index of [a,b).  The map
 * i -> phi(i) is a bijection on [0,2^B), so the minimum is attained once and
 * the argmin needs no tie-break.  An empty range (a >= b) returns k = b and
 * v = 2^B - 1 as an "invalid" marker. */
OR_EXPORT void or_rmq_scan_one(uint64_t a, uint64_t b, uint64_t r, int B,
                               uint64_t* k_out, uint64_t* v_out) {
    uint64_t bestk = b, bestv = mask_bits(B);
    int found = 0;
    for (uint64_t i = a; i < b; ++i) {
        uint64_t v = or_phi(i, r, B);
        if (!found || v < bestv) { bestv = v; bestk = i; found = 1; }
    }
    *k_out = bestk;
    *v_out = bestv;
}

/* Dyadic closed form of the same minimum.  [a,b) is cut greedily into maximal
 * aligned blocks [p, p+2^s).  Inside such a block bitrev_B(p+q) =
 * bitrev_B(p) + bitrev_s(q) * 2^(B-s) with bitrev_B(p) < 2^(B-s), so as q runs
 * over the block the shifted values run over every residue class member
 * congruent to u = (bitrev_B(p) + R) mod 2^B modulo 2^(B-s).  The block
 * minimum is therefore u mod 2^(B-s), reached where the top s bits cancel:
 * bitrev_s(q) = -(u >> (B-s)) mod 2^s.  The range minimum is the least block
 * minimum. */
OR_EXPORT void or_rmq_dyadic_one(uint64_t a, uint64_t b, uint64_t r, int B,
                                 uint64_t* k_out, uint64_t* v_out) {
    uint64_t bestk = b, bestv = mask_bits(B);
    int found = 0;
    uint64_t p = a;
    while (p < b) {
        int s = 0;
        while (s < B && (p & mask_bits(s + 1)) == 0 && p + ((uint64_t)1 << (s + 1)) <= b)
            ++s;
        uint64_t u = (or_bitrev(p, B) + r) & mask_bits(B);
        uint64_t v = u & mask_bits(B - s);
        uint64_t top = (s == 0) ? 0 : (u >> (B - s));
        uint64_t y = (((uint64_t)0) - top) & mask_bits(s);
        uint64_t x = p + (s == 0 ? 0 : or_bitrev(y, s));
        if (!found || v < bestv) { bestv = v; bestk = x; found = 1; }
        p += (uint64_t)1 << s;
    }
    *k_out = bestk;
    *v_out = bestv;
}

/* ------------------------------------------------------------------------- */
/* A tiny thread pool over index blocks: the oracle is slow per item, so it   */
/* spreads items over host cores.  Item order does not affect any result.     */
/* ------------------------------------------------------------------------- */

typedef void (*or_item_fn)(void* ctx, int64_t item);

typedef struct {
    or_item_fn fn;
    void* ctx;
    int64_t n;
    int64_t chunk;
    volatile int64_t next;
} or_pool;

static void* or_worker(void* arg) {
    or_pool* p = (or_pool*)arg;
    for (;;) {
        int64_t s = __sync_fetch_and_add(&p->next, p->chunk);
        if (s >= p->n) break;
        int64_t e = s + p->chunk < p->n ? s + p->chunk : p->n;
        for (int64_t i = s; i < e; ++i) p->fn(p->ctx, i);
    }
    return NULL;
}

static void or_parallel(or_item_fn fn, void* ctx, int64_t n, int64_t chunk, int threads) {
    or_pool p;
    p.fn = fn; p.ctx = ctx; p.n = n; p.chunk = chunk < 1 ? 1 : chunk; p.next = 0;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, or_worker, &p) == 0) ++started;
    or_worker(&p);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
}

typedef struct {
    const uint32_t *a, *b, *r;
    uint32_t *k, *v;
    int B;
    int dyadic;
} rmq_job;

static void rmq_item(void* c, int64_t q) {
    rmq_job* j = (rmq_job*)c;
    uint64_t k, v;
    if (j->dyadic) or_rmq_dyadic_one(j->a[q], j->b[q], j->r[q], j->B, &k, &v);
    else           or_rmq_scan_one(j->a[q], j->b[q], j->r[q], j->B, &k, &v);
    j->k[q] = (uint32_t)k;
    j->v[q] = (uint32_t)v;
}

/* Batched range minimum over u32 queries (B <= 32).  method 0 = scan,
 * 1 = dyadic closed form. */
OR_EXPORT void or_rmq_batch(const uint32_t* a, const uint32_t* b, const uint32_t* r,
                            int64_t n, int B, int method, uint32_t* k_out,
                            uint32_t* v_out, int threads) {
    rmq_job j = {a, b, r, k_out, v_out, B, method};
    or_parallel(rmq_item, &j, n, method ? 4096 : 16, threads);
}

/* ------------------------------------------------------------------------- */
/* Light order: Morton sort.  The paper assumes lights sorted by a spatial    */
/* hierarchy so that each leaf's position in the order is its sequence index  */
/* i (Section 1).  The order used is ascending (Morton code, original index).  */
/* ------------------------------------------------------------------------- */

/* Coordinate -> 21-bit cell index against the box [lo, hi]. */
static uint32_t or_cell(float x, float lo, float hi) {
    float u = (x - lo) / (hi - lo);
    if (!(u > 0.0f)) u = 0.0f;
    if (u > 1.0f) u = 1.0f;
    uint32_t q = (uint32_t)(u * 2097152.0f);
    return q > 2097151u ? 2097151u : q;
}

/* Bit k of the x cell goes to bit 3k+2, y to 3k+1, z to 3k. */
OR_EXPORT uint64_t or_morton(float x, float y, float z, const float* box) {
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {1.f, 1.f, 1.f};
    if (box) { lo[0] = box[0]; lo[1] = box[1]; lo[2] = box[2];
               hi[0] = box[3]; hi[1] = box[4]; hi[2] = box[5]; }
    uint32_t cx = or_cell(x, lo[0], hi[0]);
    uint32_t cy = or_cell(y, lo[1], hi[1]);
    uint32_t cz = or_cell(z, lo[2], hi[2]);
    uint64_t code = 0;
    for (int k = 0; k < 21; ++k) {
        code |= (uint64_t)((cx >> k) & 1u) << (3 * k + 2);
        code |= (uint64_t)((cy >> k) & 1u) << (3 * k + 1);
        code |= (uint64_t)((cz >> k) & 1u) << (3 * k);
    }
    return code;
}

typedef struct { uint64_t code; uint32_t id; } or_key;

static int or_key_cmp(const void* p, const void* q) {
    const or_key* x = (const or_key*)p;
    const or_key* y = (const or_key*)q;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* perm_out[i] = original index of the light that gets sequence index i. */
OR_EXPORT int or_morton_order(const float* xyz, uint32_t n, const float* box,
                              uint32_t* perm_out) {
    or_key* keys = (or_key*)malloc(sizeof(or_key) * (n ? n : 1));
    if (!keys) return -1;
    for (uint32_t i = 0; i < n; ++i) {
        keys[i].code = or_morton(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1],
                                 xyz[3 * (size_t)i + 2], box);
        keys[i].id = i;
    }
    qsort(keys, n, sizeof(or_key), or_key_cmp);
    for (uint32_t i = 0; i < n; ++i) perm_out[i] = keys[i].id;
    free(keys);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Per-eye shift and the leaf acceptance test.                                */
/* ------------------------------------------------------------------------- */

/* r_j: eye j sits at pixel (x, y) = (j mod W, j div W); its shift is the tile
 * entry at row (x mod 64), column (y mod 64), plus a request-wide offset, mod
 * 2^32 (Section 1: one Cranley-Patterson rotation per eye vertex taken from a
 * dither tile over the image plane; Section 3: an extra rotation is absorbed
 * into the shift). */
OR_EXPORT uint32_t or_eye_shift(const uint32_t* tile, uint32_t j, uint32_t width,
                                uint32_t offset) {
    uint32_t x = j % width;
    uint32_t y = j / width;
    return tile[(x % 64u) * 64u + (y % 64u)] + offset;
}

/* Extra rotation for sample n (Section 3): the rank-1 lattice
 * psi(n) = (s0 + n * alpha) mod 1 with alpha = 1/golden ratio, in 32-bit
 * fixed point with alpha rounded to the nearest multiple of 2^-32.  The
 * rounded constant is derived here from (sqrt(5) - 1) / 2 rather than typed
 * in. */
OR_EXPORT uint32_t or_golden_alpha(void) {
    double inv_phi = (sqrt(5.0) - 1.0) / 2.0;
    return (uint32_t)floor(inv_phi * 4294967296.0 + 0.5);
}

OR_EXPORT uint32_t or_psi(uint32_t n, uint32_t s0) {
    uint64_t v = (uint64_t)s0 + (uint64_t)n * (uint64_t)or_golden_alpha();
    return (uint32_t)(v & 0xFFFFFFFFull);
}

/* Acceptance probability of the pair: p = min(1, s / |e - l|^2), binary32,
 * squared distance summed as (dx^2 + dy^2) + dz^2, correctly rounded
 * division. */
OR_EXPORT float or_accept_prob(const float* e, const float* l, float s) {
    float dx = l[0] - e[0];
    float dy = l[1] - e[1];
    float dz = l[2] - e[2];
    float dx2 = dx * dx;
    float dy2 = dy * dy;
    float dz2 = dz * dz;
    float d2 = (dx2 + dy2) + dz2;
    float p = s / d2;
    return p < 1.0f ? p : 1.0f;
}

/* Russian roulette with the pair's fixed-point random number xi (32 bits):
 * keep the pair when xi / 2^32 < p.  For an integer xi that is the same as
 * xi < ceil(p * 2^32); p * 2^32 is exact in binary32 (a power-of-two scale),
 * and the comparison is done in double so nothing is rounded. */
OR_EXPORT int or_accept(const float* e, const float* l, float s, uint32_t xi) {
    float p = or_accept_prob(e, l, s);
    if (p >= 1.0f) return 1;
    double t = (double)(p * 4294967296.0f);
    return (double)xi < t;
}

/* Russian-roulette weight of a kept pair: 1 / p in binary32 (correctly
 * rounded reciprocal), the factor that keeps the culled estimator unbiased
 * (Section 1: roulette with probability p). */
OR_EXPORT float or_accept_weight(const float* e, const float* l, float s) {
    return 1.0f / or_accept_prob(e, l, s);
}

/* ------------------------------------------------------------------------- */
/* All-pairs accepted set for a selection of eyes.                            */
/* ------------------------------------------------------------------------- */

/* SplitMix64 finaliser, used only to fingerprint a set of light indices so
 * that large sets can be compared without storing them. */
static uint64_t or_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

OR_EXPORT uint64_t or_fingerprint_hash(uint64_t i) { return or_mix(i); }

typedef struct {
    const float* eyes;      /* 3 * n_eyes, eye positions by eye index j */
    const uint32_t* sel;    /* selected eye indices */
    uint32_t width, offset;
    const uint32_t* tile;
    const float* lights;    /* 3 * n_l, already in sequence (sorted) order */
    uint32_t n_l;
    float s;
    uint32_t n_samples;     /* >= 1: sample n uses the extra rotation psi(n) */
    uint32_t psi_s0;        /* lattice start s0 (used when n_samples > 1) */
    uint64_t* count;        /* per selected eye (summed over samples) */
    uint64_t* fp_sum;       /* per selected eye, optional */
    uint64_t* fp_xor;       /* per selected eye, optional */
    const uint64_t* list_off; /* per selected eye, optional: start in list */
    uint32_t* list;         /* accepted light indices (and sample ids) */
    uint32_t* list_n;       /* sample id per listed pair, optional */
} acc_job;

static void acc_item(void* c, int64_t q) {
    acc_job* J = (acc_job*)c;
    uint32_t j = J->sel[q];
    const float* e = J->eyes + 3 * (size_t)j;
    uint32_t r0 = or_eye_shift(J->tile, j, J->width, J->offset);
    uint64_t cnt = 0, fs = 0, fx = 0;
    uint64_t pos = J->list_off ? J->list_off[q] : 0;
    for (uint32_t n = 0; n < J->n_samples; ++n) {
        uint32_t r = r0 + (J->n_samples > 1 ? or_psi(n, J->psi_s0) : 0u);
        for (uint32_t i = 0; i < J->n_l; ++i) {
            uint32_t xi = (uint32_t)or_phi(i, r, 32);
            if (or_accept(e, J->lights + 3 * (size_t)i, J->s, xi)) {
                uint64_t h = or_mix(((uint64_t)n << 32) | i);
                ++cnt; fs += h; fx ^= h;
                if (J->list) {
                    J->list[pos] = i;
                    if (J->list_n) J->list_n[pos] = n;
                    ++pos;
                }
            }
        }
    }
    J->count[q] = cnt;
    if (J->fp_sum) J->fp_sum[q] = fs;
    if (J->fp_xor) J->fp_xor[q] = fx;
}

/* For each selected eye j = sel[q]: every light i (sequence order) with
 * xi_ij = (Phi_2(i) + r_j) mod 1 passing the acceptance test.  Writes counts
 * and fingerprints (sum and xor of SplitMix64 of ((n << 32) | i)); when
 * list/list_off are given, also the accepted indices in ascending i, sample by
 * sample, starting at list_off[q].  With n_samples > 1, sample n of eye j uses
 * the shift r_j + psi(n) (Section 3, the extra rotation absorbed into the
 * shift); with n_samples == 1 the shift is r_j alone. */
OR_EXPORT void or_accept_eyes(const float* eyes, const uint32_t* sel, int64_t n_sel,
                              uint32_t width, uint32_t offset, const uint32_t* tile,
                              const float* lights_sorted, uint32_t n_l, float s,
                              uint32_t n_samples, uint32_t psi_s0,
                              uint64_t* count, uint64_t* fp_sum, uint64_t* fp_xor,
                              const uint64_t* list_off, uint32_t* list,
                              uint32_t* list_n, int threads) {
    acc_job J = {eyes, sel, width, offset, tile, lights_sorted, n_l, s,
                 n_samples ? n_samples : 1, psi_s0, count, fp_sum, fp_xor,
                 list_off, list, list_n};
    or_parallel(acc_item, &J, n_sel, 1, threads);
}
