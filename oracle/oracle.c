/*
 * CPU oracle for Seismic query processing.  TEST INFRASTRUCTURE ONLY: the
 * product path never links, loads or calls this file.
 *
 * Plain, slow and direct.  It shares no code with the GPU library: it has
 * its own readers for the CSR inputs and the serialized index, its own fp16
 * decoding and its own search loop.
 *
 * What it computes:
 *   - exact sparse MIPS (Definition "Sparse MIPS", Section 1.1): the k
 *     documents with the largest inner product <q, u>, ties by doc id;
 *   - block-pruned search in the order of Algorithm 2 ("Query processing
 *     with Seismic", Section 4.5), with the kappa-NN refinement disabled;
 *   - a structural check of a serialized index against the indexing
 *     algorithm of Section 4.4 (Set alpha-MSS per column with a fixed cap,
 *     blocking by shallow K-means of Section 4.1.2, max summaries of the
 *     "summary" equation, gamma-MSS of the summaries, u8 scalar
 *     quantization of Section 4.1.3).
 *
 * Arithmetic: inputs are fp16.  Products and sums are taken in fp64.  For
 * values in [2^-6, 2^6] every product is a multiple of 2^-32 and every sum of
 * at most 400 such products stays below 2^21, so the fp64 sum is exact and
 * the result rounded once to fp32 is independent of summation order.  The
 * same holds for summary scores because the quantizer keeps m and the
 * sub-interval size on the 2^-14 grid.  or_value_range() reports whether an
 * input satisfies the range; outside it results are still computed but are
 * no longer order-independent.
 */
#include <fcntl.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

/* ------------------------------------------------------------------ fp16 */

static double half_to_double(uint16_t h) {
    int e = (h >> 10) & 0x1F;
    int f = h & 0x3FF;
    double v;
    if (e == 0) v = ldexp((double)f, -24);
    else if (e == 31) v = f ? NAN : INFINITY;
    else v = ldexp((double)(1024 + f), e - 25);
    return (h & 0x8000) ? -v : v;
}

/* fp16 value as an exact integer multiple of 2^-24 (finite, >= 0 only). */
static uint64_t half_to_units24(uint16_t h) {
    int e = (h >> 10) & 0x1F;
    uint64_t f = h & 0x3FF;
    if (e == 0) return f;
    return (1024 + f) << (e - 1);
}

static inline uint32_t w_term(uint32_t w) { return w & 0xFFFFu; }
static inline uint16_t w_half(uint32_t w) { return (uint16_t)(w >> 16); }

/* Query rows follow the library's input conventions: at most
   OR_MAX_QUERY_NNZ entries are read; a row whose terms are not strictly
   ascending (one entry per coordinate) is answered as an empty query; an
   entry with a term >= dim or a value that is not finite and positive is
   ignored. */
#define OR_MAX_QUERY_NNZ 1024

static uint64_t row_len(uint64_t n) { return n < OR_MAX_QUERY_NNZ ? n : OR_MAX_QUERY_NNZ; }

static int row_ascending(const uint32_t* w, uint64_t n) {
    for (uint64_t j = 1; j < row_len(n); ++j)
        if (w_term(w[j]) <= w_term(w[j - 1])) return 0;
    return 1;
}

static int value_ok(uint16_t h) { return (h & 0x8000) == 0 && h != 0 && ((h >> 10) & 0x1F) != 31; }

/* ------------------------------------------------------------- index file */

#define OR_MAGIC "SEISMIC"
#define OR_HEADER_BYTES 128

typedef struct {
    uint32_t dim;
    uint64_t n_docs, nnz, n_blocks, n_postings, n_summary;
    uint32_t lambda, beta;
    double gamma;
    double alpha; /* > 0: proportional caps ceil(alpha * |L_i|) (header offset 88) */
    uint64_t seed;
    uint32_t qbits;
    const uint64_t* row_ptr;
    const uint32_t* words;
    const uint32_t* list_off;
    const uint32_t* blk_post_off;
    const uint64_t* blk_sum_off;
    const float* blk_m;
    const float* blk_delta;
    const uint32_t* blk_centroid;
    const uint32_t* postings;
    const uint16_t* sum_term;
    const uint8_t* sum_code;
    /* ownership of the mapping */
    void* map;
    size_t map_len;
} or_index;

static uint64_t align64(uint64_t x) { return (x + 63) & ~(uint64_t)63; }

static int parse(or_index* ix, const uint8_t* base, uint64_t size) {
    if (size < OR_HEADER_BYTES || memcmp(base, OR_MAGIC, 7) != 0 || base[7] != 0) return -1;
    uint32_t version;
    memcpy(&version, base + 8, 4);
    if (version != 1) return -2;
    memcpy(&ix->dim, base + 12, 4);
    memcpy(&ix->n_docs, base + 16, 8);
    memcpy(&ix->nnz, base + 24, 8);
    memcpy(&ix->n_blocks, base + 32, 8);
    memcpy(&ix->n_postings, base + 40, 8);
    memcpy(&ix->n_summary, base + 48, 8);
    memcpy(&ix->lambda, base + 56, 4);
    memcpy(&ix->beta, base + 60, 4);
    memcpy(&ix->alpha, base + 88, 8);
    memcpy(&ix->gamma, base + 64, 8);
    memcpy(&ix->seed, base + 72, 8);
    memcpy(&ix->qbits, base + 80, 4);
    uint64_t off = OR_HEADER_BYTES;
    const uint8_t* p[11];
    uint64_t sz[11] = {
        8 * (ix->n_docs + 1), 4 * ix->nnz, 4 * ((uint64_t)ix->dim + 1), 4 * (ix->n_blocks + 1),
        8 * (ix->n_blocks + 1), 4 * ix->n_blocks, 4 * ix->n_blocks, 4 * ix->n_blocks,
        4 * ix->n_postings, 2 * ix->n_summary, ix->n_summary};
    for (int i = 0; i < 11; ++i) {
        off = align64(off);
        if (off + sz[i] > size) return -3;
        p[i] = base + off;
        off += sz[i];
    }
    ix->row_ptr = (const uint64_t*)p[0];
    ix->words = (const uint32_t*)p[1];
    ix->list_off = (const uint32_t*)p[2];
    ix->blk_post_off = (const uint32_t*)p[3];
    ix->blk_sum_off = (const uint64_t*)p[4];
    ix->blk_m = (const float*)p[5];
    ix->blk_delta = (const float*)p[6];
    ix->blk_centroid = (const uint32_t*)p[7];
    ix->postings = (const uint32_t*)p[8];
    ix->sum_term = (const uint16_t*)p[9];
    ix->sum_code = (const uint8_t*)p[10];
    /* offsets must be monotone and in range */
    if (ix->row_ptr[0] != 0 || ix->row_ptr[ix->n_docs] != ix->nnz) return -4;
    if (ix->list_off[0] != 0 || ix->list_off[ix->dim] != ix->n_blocks) return -4;
    if (ix->blk_post_off[0] != 0 || ix->blk_post_off[ix->n_blocks] != ix->n_postings) return -4;
    if (ix->blk_sum_off[0] != 0 || ix->blk_sum_off[ix->n_blocks] != ix->n_summary) return -4;
    for (uint64_t i = 0; i < ix->n_docs; ++i)
        if (ix->row_ptr[i] > ix->row_ptr[i + 1]) return -4;
    for (uint32_t t = 0; t < ix->dim; ++t)
        if (ix->list_off[t] > ix->list_off[t + 1]) return -4;
    for (uint64_t b = 0; b < ix->n_blocks; ++b)
        if (ix->blk_post_off[b] > ix->blk_post_off[b + 1] || ix->blk_sum_off[b] > ix->blk_sum_off[b + 1]) return -4;
    for (uint64_t i = 0; i < ix->n_postings; ++i)
        if (ix->postings[i] >= ix->n_docs) return -4;
    for (uint64_t i = 0; i < ix->n_summary; ++i)
        if (ix->sum_term[i] >= ix->dim) return -4;
    for (uint64_t i = 0; i < ix->nnz; ++i)
        if (w_term(ix->words[i]) >= ix->dim) return -4;
    return 0;
}

or_index* or_index_open(const char* path, int* err) {
    int fd = open(path, O_RDONLY);
    if (fd < 0) { if (err) *err = -10; return NULL; }
    struct stat st;
    if (fstat(fd, &st) != 0) { close(fd); if (err) *err = -10; return NULL; }
    void* m = mmap(NULL, (size_t)st.st_size, PROT_READ, MAP_PRIVATE, fd, 0);
    close(fd);
    if (m == MAP_FAILED) { if (err) *err = -11; return NULL; }
    or_index* ix = (or_index*)calloc(1, sizeof(or_index));
    int rc = parse(ix, (const uint8_t*)m, (uint64_t)st.st_size);
    if (rc != 0) { munmap(m, (size_t)st.st_size); free(ix); if (err) *err = rc; return NULL; }
    ix->map = m;
    ix->map_len = (size_t)st.st_size;
    if (err) *err = 0;
    return ix;
}

/* The buffer must outlive the handle; nothing is copied. */
or_index* or_index_from_buffer(const void* buf, uint64_t size, int* err) {
    or_index* ix = (or_index*)calloc(1, sizeof(or_index));
    int rc = parse(ix, (const uint8_t*)buf, size);
    if (rc != 0) { free(ix); if (err) *err = rc; return NULL; }
    if (err) *err = 0;
    return ix;
}

void or_index_close(or_index* ix) {
    if (!ix) return;
    if (ix->map) munmap(ix->map, ix->map_len);
    free(ix);
}

/* dim, n_docs, nnz, n_blocks, n_postings, n_summary, lambda, beta */
void or_index_info(const or_index* ix, uint64_t out[8], double* gamma) {
    out[0] = ix->dim; out[1] = ix->n_docs; out[2] = ix->nnz; out[3] = ix->n_blocks;
    out[4] = ix->n_postings; out[5] = ix->n_summary; out[6] = ix->lambda; out[7] = ix->beta;
    if (gamma) *gamma = ix->gamma;
}

/* Raw section pointers, for tests that inspect the structure with numpy. */
void or_index_sections(const or_index* ix, const void* out[11]) {
    out[0] = ix->row_ptr; out[1] = ix->words; out[2] = ix->list_off; out[3] = ix->blk_post_off;
    out[4] = ix->blk_sum_off; out[5] = ix->blk_m; out[6] = ix->blk_delta; out[7] = ix->blk_centroid;
    out[8] = ix->postings; out[9] = ix->sum_term; out[10] = ix->sum_code;
}

/* 1 if every value is finite and in [2^-6, 2^6] (the exactness range). */
int or_value_range(const uint32_t* words, uint64_t nnz) {
    for (uint64_t i = 0; i < nnz; ++i) {
        double v = half_to_double(w_half(words[i]));
        if (!(v >= 0.015625 && v <= 64.0)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ top-k */

/* H is kept sorted by (score desc, id asc); "better" is that order. */
static int better(float s1, uint32_t d1, float s2, uint32_t d2) {
    return s1 > s2 || (s1 == s2 && d1 < d2);
}

static void topk_insert(float* hs, uint32_t* hid, int* hn, int k, float s, uint32_t d) {
    int n = *hn;
    if (n == k) {
        if (!better(s, d, hs[k - 1], hid[k - 1])) return;
        n = k - 1; /* pop the minimum */
    }
    int pos = n;
    while (pos > 0 && better(s, d, hs[pos - 1], hid[pos - 1])) {
        hs[pos] = hs[pos - 1];
        hid[pos] = hid[pos - 1];
        --pos;
    }
    hs[pos] = s;
    hid[pos] = d;
    *hn = n + 1;
}

static void emit(float* out_s, uint32_t* out_id, const float* hs, const uint32_t* hid, int hn, int k) {
    for (int i = 0; i < k; ++i) {
        if (i < hn) { out_s[i] = hs[i]; out_id[i] = hid[i]; }
        else { out_s[i] = -INFINITY; out_id[i] = 0xFFFFFFFFu; }
    }
}

/* -------------------------------------------------------- exact search */

static float dot_exact(const double* qd, const uint32_t* w, uint64_t n) {
    double s = 0.0;
    for (uint64_t j = 0; j < n; ++j) s += qd[w_term(w[j])] * half_to_double(w_half(w[j]));
    return (float)s;
}

/*
 * Exact top-k by brute force over the forward rows (Definition "Sparse
 * MIPS").  Documents with a zero inner product are not results; missing
 * slots are padded with (0xFFFFFFFF, -inf).
 */
int or_exact_topk(const uint64_t* d_ptr, const uint32_t* d_words, uint64_t n_docs,
                  const uint64_t* q_ptr, const uint32_t* q_words, uint64_t nq, uint32_t dim, int k,
                  uint32_t* out_ids, float* out_scores, int nthreads) {
    if (k < 1) return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double* qd = (double*)calloc(dim, sizeof(double));
        float* hs = (float*)malloc(sizeof(float) * (size_t)k);
        uint32_t* hid = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < (int64_t)nq; ++qi) {
            const int asc = row_ascending(q_words + q_ptr[qi], q_ptr[qi + 1] - q_ptr[qi]);
            for (uint64_t j = q_ptr[qi]; j < q_ptr[qi] + row_len(q_ptr[qi + 1] - q_ptr[qi]) && asc; ++j) {
                uint32_t t = w_term(q_words[j]);
                if (t >= dim) { bad = 1; continue; }
                if (!value_ok(w_half(q_words[j]))) continue;
                qd[t] = half_to_double(w_half(q_words[j]));
            }
            int hn = 0;
            for (uint64_t d = 0; d < n_docs && asc; ++d) {
                float s = dot_exact(qd, d_words + d_ptr[d], d_ptr[d + 1] - d_ptr[d]);
                if (s > 0.0f) topk_insert(hs, hid, &hn, k, s, (uint32_t)d);
            }
            emit(out_scores + (size_t)qi * k, out_ids + (size_t)qi * k, hs, hid, hn, k);
            for (uint64_t j = q_ptr[qi]; j < q_ptr[qi + 1]; ++j) {
                uint32_t t = w_term(q_words[j]);
                if (t < dim) qd[t] = 0.0;
            }
        }
        free(qd); free(hs); free(hid);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------ pruned search */

#define OR_EXACT_SUMMARIES 1u /* r_j = <q, phi(B_j)> over full vectors (no sketch, no quantization) */
#define OR_CONTINUE 2u        /* literal "continue" on a skipped block instead of stopping the list */

#define OR_NEAR_TIE_REL 1e-5

/* ------------------------------------------------ learned block probe
 *
 * Not part of the paper: a 2-layer MLP (5 -> 64 -> 1, ReLU) that replaces
 * the heap_factor test for a cut list whose traversal starts with a full
 * heap.  Weights are 512 bf16 values: W1[64][5] (row = hidden unit), b1[64],
 * w2[64], b2, then zero padding.  Every step is defined so that the logit is
 * an exact number:
 *   - a stored weight w becomes 0 when NaN or |w| < 2^-12 and +-16 when
 *     |w| > 16;
 *   - the features of block j of cut list ci (heap full at the list's start,
 *     smallest heap score h0) are q(r_j / 16), q(r_j / h0), q(n_docs / 64),
 *     q(n_q / 64), q(ci / 8), each ratio taken in fp64 (one rounding), where
 *     q(x) is x rounded to bf16 (nearest, ties to even), then 0 below 2^-8
 *     and 16 above 16;
 *   - a_l = b1_l + sum_i W1[l][i] f_i and z = b2 + sum_l w2_l h_l with
 *     h_l = 0 for a_l <= 0, else a_l rounded to bf16, 0 below 2^-8 and 256
 *     above 256.  Every product is a multiple of 2^-34 and every sum stays
 *     below 2^19, so both sums are exact in fp64.
 * The list's blocks are visited by (z desc, block asc) and the list stops at
 * the first block with z < tau; a list that starts with a non-full heap uses
 * the heap_factor rule.  Parity unpinned by the paper (the probe is not in
 * it): pinned by its special cases in the tests. */

#define OR_PROBE_WORDS 512
#define OR_PROBE_HIDDEN 64
#define OR_PROBE_IN 5

static double bf16_value(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* x > 0 rounded to 8 significant bits, ties to even (rint in the default
   rounding mode). */
static double round_bf16(double x) {
    int e;
    double m = frexp(x, &e); /* x = m * 2^e, m in [0.5, 1) */
    return ldexp(rint(ldexp(m, 8)), e - 8);
}

static double probe_q(double x, double lo, double hi) {
    if (!(x > 0.0)) return 0.0;
    double y = round_bf16(x);
    if (y < lo) return 0.0;
    if (y > hi) return hi;
    return y;
}

static double probe_weight(uint16_t b) {
    double w = bf16_value(b);
    if (isnan(w) || fabs(w) < 0x1p-12) return 0.0;
    if (w > 16.0) return 16.0;
    if (w < -16.0) return -16.0;
    return w;
}

/* Logit of one feature vector f[5] (already quantized). */
static double probe_logit(const double* W, const double* f) {
    const double* W1 = W;
    const double* b1 = W + OR_PROBE_HIDDEN * OR_PROBE_IN;
    const double* w2 = b1 + OR_PROBE_HIDDEN;
    double z = w2[OR_PROBE_HIDDEN];
    for (int l = 0; l < OR_PROBE_HIDDEN; ++l) {
        double a = b1[l];
        for (int i = 0; i < OR_PROBE_IN; ++i) a += W1[l * OR_PROBE_IN + i] * f[i];
        z += w2[l] * probe_q(a, 0x1p-8, 256.0);
    }
    return z;
}

static void probe_features(float r, double h0, uint32_t n_docs, int n_q, int ci, double* f) {
    f[0] = probe_q((double)r / 16.0, 0x1p-8, 16.0);
    f[1] = probe_q((double)r / h0, 0x1p-8, 16.0);
    f[2] = probe_q((double)n_docs / 64.0, 0x1p-8, 16.0);
    f[3] = probe_q((double)n_q / 64.0, 0x1p-8, 16.0);
    f[4] = probe_q((double)ci / 8.0, 0x1p-8, 16.0);
}

/* Sanitized weights as fp64 (449 used values). */
static void probe_unpack(const uint16_t* probe, double* W) {
    for (int i = 0; i < OR_PROBE_WORDS; ++i) W[i] = probe_weight(probe[i]);
}

/* Quantized features and logits for explicit inputs: rows of
   (r, h0, n_docs, n_q, ci). */
int or_probe_eval(const uint16_t* probe, const float* r, const float* h0, const uint32_t* n_docs,
                  const int32_t* n_q, const int32_t* ci, uint64_t n, double* out_feat, double* out_z) {
    double W[OR_PROBE_WORDS];
    probe_unpack(probe, W);
    for (uint64_t s = 0; s < n; ++s) {
        double* f = out_feat + s * OR_PROBE_IN;
        probe_features(r[s], (double)h0[s], n_docs[s], n_q[s], ci[s], f);
        out_z[s] = probe_logit(W, f);
    }
    return 0;
}

/* The quantizers alone, for pins: mode 0 = feature q(), 1 = hidden q(),
   2 = stored-weight sanitizer (x holds bf16 bits as integers). */
void or_probe_quantize(const double* x, uint64_t n, int mode, double* out) {
    for (uint64_t i = 0; i < n; ++i) {
        if (mode == 0) out[i] = probe_q(x[i], 0x1p-8, 16.0);
        else if (mode == 1) out[i] = probe_q(x[i], 0x1p-8, 256.0);
        else out[i] = probe_weight((uint16_t)x[i]);
    }
}

typedef struct { uint32_t term; uint16_t h; double v; } qent;

/* Query cut order: value desc, then term id asc. */
static int cmp_qent(const void* a, const void* b) {
    const qent* x = (const qent*)a;
    const qent* y = (const qent*)b;
    if (x->v != y->v) return x->v > y->v ? -1 : 1;
    return (x->term > y->term) - (x->term < y->term);
}

typedef struct { float r; uint32_t j; double z; } rblk;

/* Block order: summary score desc, then block index asc. */
static int cmp_rblk(const void* a, const void* b) {
    const rblk* x = (const rblk*)a;
    const rblk* y = (const rblk*)b;
    if (x->r != y->r) return x->r > y->r ? -1 : 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* Learned order: logit desc, then block index asc. */
static int cmp_zblk(const void* a, const void* b) {
    const rblk* x = (const rblk*)a;
    const rblk* y = (const rblk*)b;
    if (x->z != y->z) return x->z > y->z ? -1 : 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* <q, S_b>: the dequantized summary value of entry e is m + code_e * delta. */
static float summary_score(const or_index* ix, const double* qd, uint64_t b) {
    double m = (double)ix->blk_m[b], delta = (double)ix->blk_delta[b];
    double s = 0.0;
    for (uint64_t e = ix->blk_sum_off[b]; e < ix->blk_sum_off[b + 1]; ++e)
        s += qd[ix->sum_term[e]] * (m + (double)ix->sum_code[e] * delta);
    return (float)s;
}

/* <q, phi(B)> with phi(B)_i = max over the block's documents (full vectors). */
static float summary_score_exact(const or_index* ix, const double* qd, uint64_t b, double* phi, uint32_t* touched) {
    int nt = 0;
    for (uint32_t p = ix->blk_post_off[b]; p < ix->blk_post_off[b + 1]; ++p) {
        uint32_t d = ix->postings[p];
        for (uint64_t j = ix->row_ptr[d]; j < ix->row_ptr[d + 1]; ++j) {
            uint32_t t = w_term(ix->words[j]);
            double v = half_to_double(w_half(ix->words[j]));
            if (phi[t] == 0.0) touched[nt++] = t;
            if (v > phi[t]) phi[t] = v;
        }
    }
    double s = 0.0;
    for (int i = 0; i < nt; ++i) { s += qd[touched[i]] * phi[touched[i]]; }
    for (int i = 0; i < nt; ++i) phi[touched[i]] = 0.0;
    return (float)s;
}

/*
 * Summary scores of one list for one query row (Algorithm 2, the summary
 * step): out[j] = r_j of the j-th block of term t's list, as the pruned
 * search computes it (the dequantized gamma-MSS summary of Section 4.1.3),
 * and, when out_exact is not NULL, out_exact[j] = <q, phi(B_j)> over the
 * full document vectors.  Returns the number of blocks, or -1 when t is out
 * of range.
 */
int or_summary_scores(const or_index* ix, const uint32_t* q_words, uint64_t q_nnz, uint32_t t,
                      float* out, float* out_exact) {
    if (t >= ix->dim) return -1;
    double* qd = (double*)calloc(ix->dim, sizeof(double));
    double* phi = (double*)calloc(ix->dim, sizeof(double));
    uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * ix->dim);
    for (uint64_t j = 0; j < row_len(q_nnz) && row_ascending(q_words, q_nnz); ++j) {
        uint32_t qt = w_term(q_words[j]);
        if (qt < ix->dim && value_ok(w_half(q_words[j]))) qd[qt] = half_to_double(w_half(q_words[j]));
    }
    uint32_t b0 = ix->list_off[t], b1 = ix->list_off[t + 1];
    for (uint32_t b = b0; b < b1; ++b) {
        out[b - b0] = summary_score(ix, qd, b);
        if (out_exact) out_exact[b - b0] = summary_score_exact(ix, qd, b, phi, touched);
    }
    free(qd); free(phi); free(touched);
    return (int)(b1 - b0);
}

/*
 * Block-pruned search, Algorithm 2 with kappa = 0:
 *   1. cut: the first min(c, n_q) query entries by (value desc, id asc);
 *      c = 0 keeps them all (stand-in for the alpha_q-MSS of the query);
 *   2. for each cut term in that order, score every block of its list by
 *      the summary inner product r_j over the full query;
 *   3. visit blocks by (r desc, block index asc); once the heap holds k
 *      documents a block with r * heap_factor < heap.min is skipped, and
 *      because r only decreases along the order and heap.min never
 *      decreases, every later block of the list is skipped too (stop);
 *   4. otherwise score every document of the block exactly and keep the k
 *      best distinct ids by (score desc, id asc).
 *
 * Outputs per query: ids/scores [k], prefix[c_cap] = evaluated blocks per
 * cut list (0 for unused slots), counters[8]:
 *   0 summary entries of the cut lists, 1 blocks of the cut lists,
 *   2 blocks evaluated, 3 documents in evaluated blocks,
 *   4 nonzeros of those documents, 5 prune tests with a full heap,
 *   6 near-tie prune tests (|r*hf - min| <= 1e-5 * min), 7 cut length.
 * With a probe (not NULL), a list that starts with a full heap is walked by
 * the learned rule instead (see the probe section above); each of its blocks
 * counts as one prune test.  out_hmin (may be NULL) receives, per cut list,
 * the smallest heap score at the list's start (-1 when the heap is not full).
 *
 * qmass > 0 shortens the cut to the alpha_q-MSS of the query (Definition
 * of alpha-MSS, Section 3.2, with alpha_q = qmass; ties by term id): the
 * first m entries of the cut order, m the smallest count whose values sum
 * to at least qmass times the query's l1 mass (fp64, exact); cut > 0 still
 * caps the count.
 *
 * kappa > 0 adds the refinement of Algorithm 2 (Section 4.5, last block)
 * with the kappa-NN graph knn[n_docs * kappa] (0xFFFFFFFF = no neighbour):
 * S = the ids in the heap after the traversal; every distinct neighbour of
 * a member of S that is not itself in S is scored exactly and offered to
 * the heap (a zero score is not a result).  Those documents are added to
 * counters 3 and 4.
 */
int or_pruned_search(const or_index* ix, const uint64_t* q_ptr, const uint32_t* q_words, uint64_t nq,
                     int k, int cut, float hf, uint32_t flags, int nthreads, int c_cap,
                     uint32_t* out_ids, float* out_scores, uint16_t* out_prefix, uint64_t* out_counters,
                     const uint16_t* probe, double tau, float* out_hmin, const uint32_t* knn, int kappa,
                     double qmass) {
    if (k < 1 || cut < 0 || !(hf > 0.0f) || c_cap < 1) return -1;
    double PW[OR_PROBE_WORDS];
    if (probe) probe_unpack(probe, PW);
    const uint32_t dim = ix->dim;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double* qd = (double*)calloc(dim, sizeof(double));
        double* phi = (double*)calloc(dim, sizeof(double));
        uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * dim);
        float* hs = (float*)malloc(sizeof(float) * (size_t)k);
        uint32_t* hid = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)k);
        qent* qe = (qent*)malloc(sizeof(qent) * (dim + 1));
        rblk* rb = NULL;
        size_t rb_cap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < (int64_t)nq; ++qi) {
            uint64_t* cnt = out_counters + (size_t)qi * 8;
            uint16_t* pref = out_prefix + (size_t)qi * c_cap;
            memset(cnt, 0, 8 * sizeof(uint64_t));
            for (int c = 0; c < c_cap; ++c) pref[c] = 0;
            if (out_hmin) for (int c = 0; c < c_cap; ++c) out_hmin[(size_t)qi * c_cap + c] = -1.0f;
            int nqe = 0;
            const int asc = row_ascending(q_words + q_ptr[qi], q_ptr[qi + 1] - q_ptr[qi]);
            for (uint64_t j = q_ptr[qi]; j < q_ptr[qi] + row_len(q_ptr[qi + 1] - q_ptr[qi]) && asc; ++j) {
                uint32_t t = w_term(q_words[j]);
                if (t >= dim) { bad = 1; continue; }
                if (!value_ok(w_half(q_words[j]))) continue;
                qe[nqe].term = t;
                qe[nqe].h = w_half(q_words[j]);
                qe[nqe].v = half_to_double(qe[nqe].h);
                qd[t] = qe[nqe].v;
                ++nqe;
            }
            qsort(qe, (size_t)nqe, sizeof(qent), cmp_qent);
            int ncut = (cut == 0 || cut > nqe) ? nqe : cut;
            if (qmass > 0.0) {
                /* alpha_q-MSS of the query (Algorithm 2, first step): the
                   shortest prefix of the value-ordered entries whose mass
                   reaches qmass * ||q||_1 */
                double total = 0.0, cum = 0.0;
                for (int j = 0; j < nqe; ++j) total += qe[j].v;
                const double target = qmass * total;
                int m = 0;
                while (m < nqe && cum < target) cum += qe[m++].v;
                if (m < ncut) ncut = m;
            }
            if (ncut > c_cap) { bad = 1; ncut = c_cap; }
            cnt[7] = (uint64_t)ncut;
            int hn = 0;
            for (int ci = 0; ci < ncut; ++ci) {
                uint32_t t = qe[ci].term;
                uint32_t b0 = ix->list_off[t], b1 = ix->list_off[t + 1];
                uint32_t nb = b1 - b0;
                if (hn == k && out_hmin) out_hmin[(size_t)qi * c_cap + ci] = hs[k - 1];
                if (nb == 0) continue;
                if (nb > rb_cap) { rb_cap = nb; rb = (rblk*)realloc(rb, sizeof(rblk) * rb_cap); }
                const int learned = probe != NULL && hn == k;
                for (uint32_t j = 0; j < nb; ++j) {
                    uint64_t b = (uint64_t)b0 + j;
                    rb[j].j = j;
                    if (flags & OR_EXACT_SUMMARIES) rb[j].r = summary_score_exact(ix, qd, b, phi, touched);
                    else rb[j].r = summary_score(ix, qd, b);
                    cnt[0] += ix->blk_sum_off[b + 1] - ix->blk_sum_off[b];
                    if (learned) {
                        double f[OR_PROBE_IN];
                        probe_features(rb[j].r, (double)hs[k - 1], ix->blk_post_off[b + 1] - ix->blk_post_off[b],
                                       nqe, ci, f);
                        rb[j].z = probe_logit(PW, f);
                    }
                }
                cnt[1] += nb;
                qsort(rb, nb, sizeof(rblk), learned ? cmp_zblk : cmp_rblk);
                if (learned) cnt[5] += nb;
                uint32_t evaluated = 0;
                for (uint32_t pos = 0; pos < nb; ++pos) {
                    uint64_t b = (uint64_t)b0 + rb[pos].j;
                    if (learned) {
                        if (rb[pos].z < tau) break;
                    } else if (hn == k) {
                        double lhs = (double)rb[pos].r * (double)hf;
                        double hmin = (double)hs[k - 1];
                        cnt[5]++;
                        if (fabs(lhs - hmin) <= OR_NEAR_TIE_REL * hmin) cnt[6]++;
                        if (lhs < hmin) {
                            if (flags & OR_CONTINUE) continue;
                            break;
                        }
                    }
                    evaluated++;
                    cnt[2]++;
                    for (uint32_t p = ix->blk_post_off[b]; p < ix->blk_post_off[b + 1]; ++p) {
                        uint32_t d = ix->postings[p];
                        uint64_t r0 = ix->row_ptr[d], r1 = ix->row_ptr[d + 1];
                        cnt[3]++;
                        cnt[4] += r1 - r0;
                        int in_heap = 0;
                        for (int h = 0; h < hn; ++h) if (hid[h] == d) { in_heap = 1; break; }
                        if (in_heap) continue; /* the heap holds distinct ids */
                        float s = dot_exact(qd, ix->words + r0, r1 - r0);
                        topk_insert(hs, hid, &hn, k, s, d);
                    }
                }
                pref[ci] = (uint16_t)(evaluated > 65535 ? 65535 : evaluated);
            }
            if (kappa > 0 && knn) {
                /* expanded set: neighbours of the heap's members, each once */
                int ns = hn;
                uint32_t* S = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(ns > 0 ? ns : 1));
                uint32_t* cand = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(ns * kappa + 1));
                for (int h = 0; h < ns; ++h) S[h] = hid[h];
                int nc = 0;
                for (int h = 0; h < ns; ++h)
                    for (int j = 0; j < kappa; ++j) {
                        uint32_t v = knn[(size_t)S[h] * kappa + j];
                        if (v == 0xFFFFFFFFu || v >= ix->n_docs) continue;
                        int seen = 0;
                        for (int x = 0; x < ns && !seen; ++x) seen = S[x] == v;
                        for (int x = 0; x < nc && !seen; ++x) seen = cand[x] == v;
                        if (!seen) cand[nc++] = v;
                    }
                for (int c = 0; c < nc; ++c) {
                    uint32_t d = cand[c];
                    uint64_t r0 = ix->row_ptr[d], r1 = ix->row_ptr[d + 1];
                    cnt[3]++;
                    cnt[4] += r1 - r0;
                    float sc = dot_exact(qd, ix->words + r0, r1 - r0);
                    if (sc > 0.0f) topk_insert(hs, hid, &hn, k, sc, d);
                }
                free(S);
                free(cand);
            }
            emit(out_scores + (size_t)qi * k, out_ids + (size_t)qi * k, hs, hid, hn, k);
            for (int j = 0; j < nqe; ++j) qd[qe[j].term] = 0.0;
        }
        free(qd); free(phi); free(touched); free(hs); free(hid); free(qe); free(rb);
    }
    return bad ? -2 : 0;
}

/* ---------------------------------------------------- index structure */

typedef struct { uint32_t id; uint32_t pos; uint64_t v; } ent;

/* Value desc, then id asc: the order of Set alpha-MSS columns (ids are
   document ids) and of alpha-MSS (ids are coordinates). */
static int cmp_ent_val(const void* a, const void* b) {
    const ent* x = (const ent*)a;
    const ent* y = (const ent*)b;
    if (x->v != y->v) return x->v > y->v ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int cmp_ent_id(const void* a, const void* b) {
    const ent* x = (const ent*)a;
    const ent* y = (const ent*)b;
    return (x->id > y->id) - (x->id < y->id);
}

/* keep[pos] = 1 for the first m sorted entries. */
static void mark_prefix(uint64_t n, const ent* sorted, uint64_t m, uint8_t* keep) {
    for (uint64_t i = 0; i < n; ++i) keep[i] = 0;
    for (uint64_t r = 0; r < m; ++r) keep[sorted[r].pos] = 1;
}

/*
 * Set alpha-MSS, one column (Definition "Set alpha-MSS", Section 3.4): keep
 * the lambda largest values of the column; ties by id ascending.
 * keep[i] = 1 for kept entries.  Ids must be distinct.
 */
int or_column_keep(const uint32_t* ids, const uint16_t* h, uint64_t n, uint64_t lambda, uint8_t* keep) {
    ent* e = (ent*)malloc(sizeof(ent) * (n ? n : 1));
    for (uint64_t i = 0; i < n; ++i) { e[i].id = ids[i]; e[i].pos = (uint32_t)i; e[i].v = half_to_units24(h[i]); }
    qsort(e, (size_t)n, sizeof(ent), cmp_ent_val);
    mark_prefix(n, e, n < lambda ? n : lambda, keep);
    free(e);
    return 0;
}

/*
 * alpha-MSS (Definition "alpha-mass subvector sketch", Section 3.3): sort the
 * entries by value desc (ties: id asc) and keep the shortest prefix whose
 * l1 mass reaches alpha times the total (sums in fp64, exact for fp16
 * inputs).  keep[i] = 1 for kept entries; returns the number kept.
 */
int or_alpha_mss(const uint32_t* ids, const uint16_t* h, uint64_t n, double alpha, uint8_t* keep) {
    ent* e = (ent*)malloc(sizeof(ent) * (n ? n : 1));
    double total = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        e[i].id = ids[i];
        e[i].pos = (uint32_t)i;
        e[i].v = half_to_units24(h[i]);
        total += half_to_double(h[i]);
    }
    qsort(e, (size_t)n, sizeof(ent), cmp_ent_val);
    double need = alpha * total, cum = 0.0;
    uint64_t kept = 0;
    while (kept < n) {
        cum += (double)e[kept].v * 0x1p-24;
        kept++;
        if (cum >= need) break;
    }
    mark_prefix(n, e, kept, keep);
    free(e);
    return (int)kept;
}

/*
 * u8 scalar quantization of a summary (Section 4.1.3): subtract the minimum
 * m, split the range into 256 sub-intervals of equal size, store the index
 * of the sub-interval; reconstruction is m + code * size.  Reading taken
 * here: m is rounded down and the size rounded up to the 2^-14 grid (so the
 * 256 sub-intervals still cover [min, max]); the code is the floor index,
 * clamped to 255; a zero range gives size 0 and code 0.  Integer arithmetic
 * on exact multiples of 2^-24.
 */
int or_quantize(const uint16_t* h, uint64_t n, float* m_out, float* delta_out, uint8_t* codes) {
    if (n == 0) { *m_out = 0.0f; *delta_out = 0.0f; return 0; }
    uint64_t vmin = UINT64_MAX, vmax = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t v = half_to_units24(h[i]);
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
    }
    const uint64_t grid = 1024; /* 2^-14 in units of 2^-24 */
    uint64_t m_u = (vmin / grid) * grid;
    uint64_t range = vmax - m_u;
    uint64_t d_u = ((range + 256 * grid - 1) / (256 * grid)) * grid;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t c = d_u ? (half_to_units24(h[i]) - m_u) / d_u : 0;
        codes[i] = (uint8_t)(c > 255 ? 255 : c);
    }
    *m_out = (float)((double)m_u * 0x1p-24);
    *delta_out = (float)((double)d_u * 0x1p-24);
    return 0;
}

static double doc_dot_doc(const or_index* ix, uint32_t a, uint32_t b) {
    /* merge of two term-sorted rows */
    uint64_t i = ix->row_ptr[a], ie = ix->row_ptr[a + 1];
    uint64_t j = ix->row_ptr[b], je = ix->row_ptr[b + 1];
    double s = 0.0;
    while (i < ie && j < je) {
        uint32_t ti = w_term(ix->words[i]), tj = w_term(ix->words[j]);
        if (ti == tj) {
            s += half_to_double(w_half(ix->words[i])) * half_to_double(w_half(ix->words[j]));
            ++i; ++j;
        } else if (ti < tj) ++i;
        else ++j;
    }
    return s;
}

#define FAIL(...) do { snprintf(msg, (size_t)msglen, __VA_ARGS__); failed = 1; goto done; } while (0)

/*
 * Check a serialized index against the indexing algorithm of Section 4.4
 * with a fixed list cap lambda, or the proportional cap ceil(alpha * |L_i|)
 * (at most lambda) when the header's alpha is > 0.  Returns 0 when every
 * check passes, 1 with a message otherwise.
 *   - list i holds the min(|L_i|, cap_i) largest values of column i
 *     (value desc, doc id asc);
 *   - its blocks partition that list: at least 1 and at most
 *     max(1, ceil(beta * n_i / lambda)) of them, none empty, doc ids
 *     ascending inside a block, each block's centroid a member of the list;
 *   - check_clustering != 0: every document sits in the block of a centroid
 *     maximizing <u, mu> over the list's centroids (lowest block index on
 *     ties) - this costs as much as the clustering;
 *   - each summary is the gamma-MSS of the max vector phi(B) over the full
 *     document vectors, stored by term id and quantized as in or_quantize.
 * term_stride > 1 checks every term_stride-th term only.
 */
int or_check_index(const or_index* ix, int check_clustering, int term_stride, char* msg, int msglen) {
    const uint32_t dim = ix->dim;
    int failed = 0;
    msg[0] = 0;
    if (term_stride < 1) term_stride = 1;
    /* transpose the forward index */
    uint64_t* cnt = (uint64_t*)calloc((size_t)dim + 1, sizeof(uint64_t));
    for (uint64_t i = 0; i < ix->nnz; ++i) cnt[w_term(ix->words[i]) + 1]++;
    for (uint32_t t = 0; t < dim; ++t) cnt[t + 1] += cnt[t];
    uint32_t* col_id = (uint32_t*)malloc(sizeof(uint32_t) * (ix->nnz ? ix->nnz : 1));
    uint16_t* col_h = (uint16_t*)malloc(sizeof(uint16_t) * (ix->nnz ? ix->nnz : 1));
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)dim + 1));
    memcpy(fill, cnt, sizeof(uint64_t) * ((size_t)dim + 1));
    for (uint64_t d = 0; d < ix->n_docs; ++d)
        for (uint64_t j = ix->row_ptr[d]; j < ix->row_ptr[d + 1]; ++j) {
            uint32_t t = w_term(ix->words[j]);
            col_id[fill[t]] = (uint32_t)d;
            col_h[fill[t]] = w_half(ix->words[j]);
            fill[t]++;
        }
    uint8_t* seen = (uint8_t*)calloc(ix->n_docs ? ix->n_docs : 1, 1);
    uint16_t* phi = (uint16_t*)calloc(dim, sizeof(uint16_t)); /* positive fp16: bit order = value order */
    uint32_t* s_ids = (uint32_t*)malloc(sizeof(uint32_t) * dim);
    uint16_t* s_h = (uint16_t*)malloc(sizeof(uint16_t) * dim);
    uint8_t* s_keep = (uint8_t*)malloc(dim);
    ent* s_ent = (ent*)malloc(sizeof(ent) * dim);
    uint16_t* k_h = (uint16_t*)malloc(sizeof(uint16_t) * dim);
    uint8_t* k_code = (uint8_t*)malloc(dim);
    uint8_t* keep = NULL;
    size_t keep_cap = 0;
    for (uint32_t t = 0; t < dim; t += (uint32_t)term_stride) {
        uint64_t n_full = cnt[t + 1] - cnt[t];
        uint32_t b0 = ix->list_off[t], b1 = ix->list_off[t + 1];
        uint32_t nb = b1 - b0;
        if (keep_cap < n_full) { keep_cap = n_full; keep = (uint8_t*)realloc(keep, keep_cap); }
        /* the column's cap: lambda, and with alpha > 0 ceil(alpha * |L_i|)
           (Set alpha-MSS, Section 3.4), at least 1 */
        uint64_t cap = ix->lambda;
        if (ix->alpha > 0.0) {
            double c = ceil(ix->alpha * (double)n_full);
            uint64_t pc = c < 1.0 ? 1 : (uint64_t)c;
            if (pc < cap) cap = pc;
        }
        or_column_keep(col_id + cnt[t], col_h + cnt[t], n_full, cap, keep);
        uint64_t n = n_full < cap ? n_full : cap;
        if (n == 0) {
            if (nb != 0) FAIL("term %u: empty list has %u blocks", t, nb);
            continue;
        }
        uint64_t max_nb = ((uint64_t)ix->beta * n + ix->lambda - 1) / ix->lambda;
        if (max_nb < 1) max_nb = 1;
        if (nb < 1 || nb > max_nb) FAIL("term %u: %u blocks, allowed 1..%llu", t, nb, (unsigned long long)max_nb);
        uint64_t tot = 0;
        for (uint32_t b = b0; b < b1; ++b) {
            uint32_t p0 = ix->blk_post_off[b], p1 = ix->blk_post_off[b + 1];
            if (p1 == p0) FAIL("term %u block %u: empty", t, b);
            for (uint32_t p = p0 + 1; p < p1; ++p)
                if (ix->postings[p] <= ix->postings[p - 1]) FAIL("term %u block %u: doc ids not ascending", t, b);
            tot += p1 - p0;
        }
        if (tot != n) FAIL("term %u: blocks hold %llu docs, truncated list has %llu", t, (unsigned long long)tot, (unsigned long long)n);
        for (uint64_t i = 0; i < n_full; ++i) if (keep[i]) seen[col_id[cnt[t] + i]] = 1;
        for (uint32_t b = b0; b < b1; ++b)
            if (seen[ix->blk_centroid[b]] != 1) FAIL("term %u block %u: centroid %u not in the list", t, b, ix->blk_centroid[b]);
        for (uint32_t b = b0; b < b1; ++b)
            for (uint32_t p = ix->blk_post_off[b]; p < ix->blk_post_off[b + 1]; ++p) {
                uint32_t d = ix->postings[p];
                if (seen[d] != 1) FAIL("term %u: doc %u in block %u is not in the truncated list or repeats", t, d, b);
                seen[d] = 2;
            }
        for (uint64_t i = 0; i < n_full; ++i) seen[col_id[cnt[t] + i]] = 0;
        if (check_clustering) {
            for (uint32_t b = b0; b < b1; ++b)
                for (uint32_t p = ix->blk_post_off[b]; p < ix->blk_post_off[b + 1]; ++p) {
                    uint32_t d = ix->postings[p];
                    double own = doc_dot_doc(ix, d, ix->blk_centroid[b]);
                    for (uint32_t o = b0; o < b1; ++o) {
                        if (o == b) continue;
                        double other = doc_dot_doc(ix, d, ix->blk_centroid[o]);
                        if (other > own || (other == own && o < b))
                            FAIL("term %u: doc %u assigned to block %u but the centroid of block %u scores %.17g vs %.17g",
                                 t, d, b, o, other, own);
                    }
                }
        }
        for (uint32_t b = b0; b < b1; ++b) {
            /* phi(B)_i = max over the block's documents (summary equation) */
            int nt = 0;
            for (uint32_t p = ix->blk_post_off[b]; p < ix->blk_post_off[b + 1]; ++p) {
                uint32_t d = ix->postings[p];
                for (uint64_t j = ix->row_ptr[d]; j < ix->row_ptr[d + 1]; ++j) {
                    uint32_t tt = w_term(ix->words[j]);
                    uint16_t h = w_half(ix->words[j]);
                    if (phi[tt] == 0) s_ids[nt++] = tt;
                    if (h > phi[tt]) phi[tt] = h;
                }
            }
            for (int i = 0; i < nt; ++i) { s_h[i] = phi[s_ids[i]]; phi[s_ids[i]] = 0; }
            int kept = or_alpha_mss(s_ids, s_h, (uint64_t)nt, ix->gamma, s_keep);
            uint64_t s0 = ix->blk_sum_off[b], s1 = ix->blk_sum_off[b + 1];
            if ((uint64_t)kept != s1 - s0)
                FAIL("term %u block %u: summary has %llu entries, gamma-MSS has %d", t, b, (unsigned long long)(s1 - s0), kept);
            int nk = 0;
            for (int i = 0; i < nt; ++i) if (s_keep[i]) { s_ent[nk].id = s_ids[i]; s_ent[nk].v = s_h[i]; nk++; }
            qsort(s_ent, (size_t)nk, sizeof(ent), cmp_ent_id);
            for (int i = 0; i < nk; ++i) k_h[i] = (uint16_t)s_ent[i].v;
            float m_f, d_f;
            or_quantize(k_h, (uint64_t)nk, &m_f, &d_f, k_code);
            if (ix->blk_m[b] != m_f || ix->blk_delta[b] != d_f)
                FAIL("term %u block %u: (m, delta) = (%.9g, %.9g), expected (%.9g, %.9g)", t, b, ix->blk_m[b], ix->blk_delta[b], m_f, d_f);
            for (int i = 0; i < nk; ++i)
                if (ix->sum_term[s0 + (uint64_t)i] != s_ent[i].id || ix->sum_code[s0 + (uint64_t)i] != k_code[i])
                    FAIL("term %u block %u entry %d: (term, code) = (%u, %u), expected (%u, %u)", t, b, i,
                         ix->sum_term[s0 + (uint64_t)i], ix->sum_code[s0 + (uint64_t)i], s_ent[i].id, k_code[i]);
        }
    }
done:
    free(cnt); free(col_id); free(col_h); free(fill); free(seen); free(phi);
    free(s_ids); free(s_h); free(s_keep); free(s_ent); free(k_h); free(k_code); free(keep);
    return failed;
}
