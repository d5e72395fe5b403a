/*
 * Seeded synthetic sparse-vector generator.
 *
 * Produces CSR matrices shaped like learned-sparse-embedding corpora
 * (SPLADE-style: ~30k-term vocabulary, heavy-headed term frequencies,
 * positive fp16 weights).  This module holds no arithmetic of the search
 * method; it only draws inputs.  Both the CPU oracle and the GPU library
 * consume its output.
 *
 * Row law (one definition for every workload):
 *   - number of nonzeros n: Poisson(mean) clipped to [lo, hi], or uniform
 *     integer in [lo, hi];
 *   - coordinate ids: successive i.i.d. draws of a rank r in [1, dim] with
 *     P(r) proportional to r^-s (term id = r - 1), duplicates discarded,
 *     until n distinct ids are collected; ids stored ascending;
 *   - values: exp(sigma * z), z standard normal (Box-Muller), clamped to
 *     [2^-6, 2^6] and rounded to IEEE binary16 (round to nearest even).
 *     The clamp sits ~6.9 standard deviations out for sigma = 0.6.
 *
 * Randomness: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), key = (seed, stream), counter =
 * (row, block).  Every row's draws depend only on (seed, stream, row), so
 * the output is identical for any thread count.
 *
 * Storage: row_ptr u64[n_rows + 1]; word u32 = term | (fp16 bits << 16).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void synth_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0; k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int used;
} rng_t;

static void rng_init(rng_t* g, uint64_t seed, uint32_t stream, uint64_t row) {
    g->key[0] = (uint32_t)seed ^ (uint32_t)(seed >> 32);
    g->key[1] = stream;
    g->ctr[0] = (uint32_t)row;
    g->ctr[1] = (uint32_t)(row >> 32);
    g->ctr[2] = 0;
    g->ctr[3] = 0;
    g->used = 4;
}

static uint32_t rng_u32(rng_t* g) {
    if (g->used == 4) {
        synth_philox4x32_10(g->ctr, g->key, g->buf);
        g->ctr[2]++;
        if (g->ctr[2] == 0) g->ctr[3]++;
        g->used = 0;
    }
    return g->buf[g->used++];
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_unif(rng_t* g) {
    uint32_t a = rng_u32(g) >> 5, b = rng_u32(g) >> 6;
    return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

/* IEEE binary16 from double, round to nearest even; input finite, >= 0.
 * Works on the double's bit fields: the 52-bit fraction is cut to 10 bits
 * (normal results) or to a multiple of 2^-24 (subnormal results), and the
 * discarded bits decide the rounding, ties to the even result. */
uint16_t synth_half_from_double(double x) {
    if (!(x > 0.0)) return 0;
    if (x >= 65520.0) return 0x7C00; /* overflow to +inf */
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    const int e = (int)((b >> 52) & 0x7FF) - 1023; /* x = 1.f * 2^e (x is a normal double here) */
    const uint64_t sig = (b & 0xFFFFFFFFFFFFFull) | (1ull << 52); /* 53-bit significand */
    int shift;      /* bits of sig below the kept unit */
    uint32_t base;  /* exponent field of the result before rounding */
    if (e >= -14) {
        shift = 42;
        base = (uint32_t)(e + 15);
    } else {
        /* subnormal: units of 2^-24, i.e. sig >> (52 - (e + 24)) */
        shift = 52 - (e + 24);
        base = 0;
        if (shift > 63) return 0; /* below 2^-25 rounds to zero */
    }
    uint64_t kept = sig >> shift;
    const uint64_t rem = sig & ((1ull << shift) - 1), half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (kept & 1))) ++kept;
    if (base == 0) return (uint16_t)kept; /* 1024 rolls into the smallest normal */
    /* kept in [1024, 2048]: implicit bit plus 10 fraction bits */
    uint32_t biased = base, mant = (uint32_t)kept - 1024;
    if (mant == 1024) { mant = 0; biased++; }
    if (biased >= 31) return 0x7C00;
    return (uint16_t)((biased << 10) | mant);
}

/* Ascending sort of n distinct 16-bit ids: two stable byte passes. */
static void sort_u16(uint16_t* a, int n, uint16_t* tmp) {
    int cnt[257];
    for (int pass = 0; pass < 2; ++pass) {
        const int sh = 8 * pass;
        memset(cnt, 0, sizeof cnt);
        for (int i = 0; i < n; ++i) cnt[((a[i] >> sh) & 0xFF) + 1]++;
        for (int i = 0; i < 256; ++i) cnt[i + 1] += cnt[i];
        for (int i = 0; i < n; ++i) tmp[cnt[(a[i] >> sh) & 0xFF]++] = a[i];
        memcpy(a, tmp, sizeof(uint16_t) * (size_t)n);
    }
}

#define GUIDE_N 65536

typedef struct {
    int dim;
    double* zipf_cdf; /* cdf[r-1] = P(rank <= r) */
    int* zipf_guide;  /* guide[k] = smallest index with cdf > k / GUIDE_N (k <= GUIDE_N) */
    int law;          /* 0 = Poisson(mean) clipped, 1 = uniform integer */
    int lo, hi;
    int pois_n;       /* table length */
    double* pois_cdf; /* cdf[n] = P(N <= n) */
    double sigma;
} law_t;

static int draw_count(const law_t* L, rng_t* g) {
    double u = rng_unif(g);
    int n;
    if (L->law == 1) {
        n = L->lo + (int)(u * (double)(L->hi - L->lo + 1));
        if (n > L->hi) n = L->hi;
        return n;
    }
    /* inversion: smallest n with cdf[n] > u */
    int a = 0, b = L->pois_n - 1;
    if (!(L->pois_cdf[b] > u)) n = b;
    else {
        while (a < b) {
            int mid = (a + b) >> 1;
            if (L->pois_cdf[mid] > u) b = mid; else a = mid + 1;
        }
        n = a;
    }
    if (n < L->lo) n = L->lo;
    if (n > L->hi) n = L->hi;
    return n;
}

/* Inversion of the Zipf cdf: the smallest index with cdf > u.  The guide
 * table narrows the search to [guide[k], guide[k + 1]] for u in
 * [k / GUIDE_N, (k + 1) / GUIDE_N); the result is the plain binary search's. */
static int draw_rank0(const law_t* L, rng_t* g) {
    double u = rng_unif(g);
    const int k = (int)(u * (double)GUIDE_N);
    int a = L->zipf_guide[k], b = L->zipf_guide[k + 1];
    while (a < b) {
        int mid = (a + b) >> 1;
        if (L->zipf_cdf[mid] > u) b = mid; else a = mid + 1;
    }
    return a; /* term id = rank - 1 */
}

static double draw_value(const law_t* L, rng_t* g) {
    double u1 = 1.0 - rng_unif(g); /* (0, 1] */
    double u2 = rng_unif(g);
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double v = exp(L->sigma * z);
    if (v < 0.015625) v = 0.015625;
    if (v > 64.0) v = 64.0;
    return v;
}

static int law_setup(law_t* L, int dim, double zipf_s, int law, double mean, int lo, int hi, double sigma) {
    L->dim = dim; L->law = law; L->lo = lo; L->hi = hi; L->sigma = sigma;
    L->zipf_cdf = (double*)malloc(sizeof(double) * (size_t)dim);
    L->zipf_guide = NULL;
    L->pois_cdf = NULL; L->pois_n = 0;
    if (!L->zipf_cdf) return -1;
    double tot = 0.0;
    for (int r = 1; r <= dim; ++r) tot += pow((double)r, -zipf_s);
    double c = 0.0;
    for (int r = 1; r <= dim; ++r) { c += pow((double)r, -zipf_s) / tot; L->zipf_cdf[r - 1] = c; }
    L->zipf_cdf[dim - 1] = 1.0;
    L->zipf_guide = (int*)malloc(sizeof(int) * (GUIDE_N + 1));
    if (!L->zipf_guide) return -1;
    for (int k = 0, a = 0; k <= GUIDE_N; ++k) {
        const double u = (double)k / (double)GUIDE_N;
        while (a < dim - 1 && !(L->zipf_cdf[a] > u)) ++a;
        L->zipf_guide[k] = a;
    }
    if (law == 0) {
        int n = hi + 1;
        L->pois_n = n;
        L->pois_cdf = (double*)malloc(sizeof(double) * (size_t)n);
        if (!L->pois_cdf) return -1;
        /* pmf via logs to avoid overflow */
        double acc = 0.0;
        for (int i = 0; i < n; ++i) {
            double lp = -mean + i * log(mean) - lgamma((double)i + 1.0);
            acc += exp(lp);
            L->pois_cdf[i] = acc;
        }
    }
    return 0;
}

static void law_free(law_t* L) { free(L->zipf_cdf); free(L->zipf_guide); free(L->pois_cdf); }

/* Pass 1: number of nonzeros of rows row0 .. row0 + n_rows - 1. */
int synth_counts_range(uint64_t row0, uint64_t n_rows, int dim, double zipf_s, int law, double mean, int lo,
                       int hi, uint64_t seed, uint32_t stream, uint32_t* counts) {
    law_t L;
    if (dim < 1 || dim > 65536 || lo < 1 || hi < lo || hi > dim) return -1;
    if (law_setup(&L, dim, zipf_s, law, mean, lo, hi, 0.6) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n_rows; ++i) {
        rng_t g;
        rng_init(&g, seed, stream, row0 + (uint64_t)i);
        counts[i] = (uint32_t)draw_count(&L, &g);
    }
    law_free(&L);
    return 0;
}

int synth_counts(uint64_t n_rows, int dim, double zipf_s, int law, double mean, int lo, int hi,
                 uint64_t seed, uint32_t stream, uint32_t* counts) {
    return synth_counts_range(0, n_rows, dim, zipf_s, law, mean, lo, hi, seed, stream, counts);
}

/* Pass 2: fill rows row0 .. row0 + n_rows - 1; row_ptr (n_rows + 1 entries,
 * relative to words) must already hold the prefix sums of their counts. */
int synth_fill_range(uint64_t row0, uint64_t n_rows, int dim, double zipf_s, int law, double mean, int lo, int hi,
                     double sigma, uint64_t seed, uint32_t stream, const uint64_t* row_ptr, uint32_t* words) {
    law_t L;
    if (dim < 1 || dim > 65536 || lo < 1 || hi < lo || hi > dim) return -1;
    if (law_setup(&L, dim, zipf_s, law, mean, lo, hi, sigma) != 0) return -1;
    int err = 0;
#pragma omp parallel
    {
        uint8_t* seen = (uint8_t*)calloc((size_t)dim, 1);
        uint16_t* ids = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(hi + 1));
        uint16_t* tmp = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(hi + 1));
        if (!seen || !ids || !tmp) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < (int64_t)n_rows; ++i) {
                rng_t g;
                rng_init(&g, seed, stream, row0 + (uint64_t)i);
                int n = draw_count(&L, &g);
                if ((uint64_t)n != row_ptr[i + 1] - row_ptr[i]) {
#pragma omp atomic write
                    err = 2;
                    continue;
                }
                int got = 0;
                while (got < n) {
                    int t = draw_rank0(&L, &g);
                    if (!seen[t]) { seen[t] = 1; ids[got++] = (uint16_t)t; }
                }
                sort_u16(ids, n, tmp);
                uint32_t* w = words + row_ptr[i];
                for (int j = 0; j < n; ++j) {
                    seen[ids[j]] = 0;
                    uint16_t h = synth_half_from_double(draw_value(&L, &g));
                    w[j] = (uint32_t)ids[j] | ((uint32_t)h << 16);
                }
            }
        }
        free(seen);
        free(ids);
        free(tmp);
    }
    law_free(&L);
    return err ? -err : 0;
}

int synth_fill(uint64_t n_rows, int dim, double zipf_s, int law, double mean, int lo, int hi, double sigma,
               uint64_t seed, uint32_t stream, const uint64_t* row_ptr, uint32_t* words) {
    return synth_fill_range(0, n_rows, dim, zipf_s, law, mean, lo, hi, sigma, seed, stream, row_ptr, words);
}
