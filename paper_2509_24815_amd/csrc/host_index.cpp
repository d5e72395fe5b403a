// Host side of libseismic: errors, threads, input validation, the index
// builder of Section 4.4 and the serialized format.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <numeric>

#include "internal.h"

void device_index_free(DeviceIndex* d);          // device.hip
int device_index_layout(const DeviceIndex* d);  // 0 none, 1 resident, 2 with block-major copies of every list, 3 of some

namespace seismic {

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

// --------------------------------------------------------------- threads

int resolve_threads(int requested) {
    if (requested > 0) return requested;
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)hc : 1;
}

void parallel_for(int64_t n, int nthreads, int64_t chunk, const std::function<void(int64_t, int)>& fn) {
    nthreads = resolve_threads(nthreads);
    if (chunk < 1) chunk = 1;
    if (nthreads == 1 || n <= chunk) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    auto worker = [&](int tid) {
        for (;;) {
            int64_t a = next.fetch_add(chunk);
            if (a >= n) break;
            int64_t b = std::min(n, a + chunk);
            for (int64_t i = a; i < b; ++i) fn(i, tid);
        }
    };
    std::vector<std::thread> ts;
    for (int t = 1; t < nthreads; ++t) ts.emplace_back(worker, t);
    worker(0);
    for (auto& t : ts) t.join();
}

// ------------------------------------------------------------ validation

int validate_csr_host(const seismic_csr* m, uint32_t max_row_nnz, const char* what) {
    if (!m) return fail(SEISMIC_EINVAL, "%s: null matrix", what);
    if (m->on_device) return fail(SEISMIC_EINVAL, "%s: host-resident rows required", what);
    if (m->dim < 1 || m->dim > 65536) return fail(SEISMIC_EINVAL, "%s: dim %u outside [1, 65536]", what, m->dim);
    if (!m->row_ptr) return fail(SEISMIC_EINVAL, "%s: null row_ptr", what);
    if (m->nnz && !m->words) return fail(SEISMIC_EINVAL, "%s: null words", what);
    if (m->row_ptr[0] != 0 || m->row_ptr[m->n_rows] != m->nnz)
        return fail(SEISMIC_EINVAL, "%s: row_ptr must start at 0 and end at nnz", what);
    std::atomic<int64_t> bad_row{-1};
    std::atomic<int> bad_kind{0};
    parallel_for((int64_t)m->n_rows, 0, 4096, [&](int64_t i, int) {
        uint64_t a = m->row_ptr[i], b = m->row_ptr[i + 1];
        int kind = 0;
        if (b < a || b > m->nnz) kind = 1;
        else if (b - a > max_row_nnz) kind = 2;
        else {
            for (uint64_t j = a; j < b && !kind; ++j) {
                uint32_t t = word_term(m->words[j]);
                if (t >= m->dim) kind = 3;
                else if (j > a && t <= word_term(m->words[j - 1])) kind = 4;
                else if (!half_positive_finite(word_half(m->words[j]))) kind = 5;
            }
        }
        if (kind) { bad_kind.store(kind); bad_row.store(i); }
    });
    if (bad_kind.load()) {
        static const char* why[] = {"", "row_ptr not monotone", "row too long", "term id >= dim",
                                    "terms not strictly ascending", "value not finite and positive"};
        return fail(SEISMIC_EINVAL, "%s: row %lld: %s", what, (long long)bad_row.load(), why[bad_kind.load()]);
    }
    return SEISMIC_OK;
}

// ------------------------------------------------------------------- CSC

void build_csc(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs, uint32_t dim, int nthreads,
               HostCSC& out) {
    nthreads = resolve_threads(nthreads);
    const uint64_t nnz = row_ptr[n_docs];
    int nch = (int)std::min<uint64_t>((uint64_t)nthreads * 4, std::max<uint64_t>(1, n_docs));
    std::vector<uint64_t> bounds(nch + 1);
    for (int c = 0; c <= nch; ++c) bounds[c] = n_docs * (uint64_t)c / (uint64_t)nch;
    // counts[c][t]
    std::vector<uint64_t> counts((size_t)nch * (dim + 1), 0);
    parallel_for(nch, nthreads, 1, [&](int64_t c, int) {
        uint64_t* cnt = counts.data() + (size_t)c * (dim + 1);
        for (uint64_t j = row_ptr[bounds[c]]; j < row_ptr[bounds[c + 1]]; ++j) cnt[word_term(words[j])]++;
    });
    out.off.assign((size_t)dim + 1, 0);
    // offsets: term-major, chunk-minor so every term stays doc-ascending
    uint64_t run = 0;
    for (uint32_t t = 0; t < dim; ++t) {
        out.off[t] = run;
        for (int c = 0; c < nch; ++c) {
            uint64_t v = counts[(size_t)c * (dim + 1) + t];
            counts[(size_t)c * (dim + 1) + t] = run;
            run += v;
        }
    }
    out.off[dim] = run;
    out.doc.resize(nnz);
    out.val.resize(nnz);
    parallel_for(nch, nthreads, 1, [&](int64_t c, int) {
        uint64_t* pos = counts.data() + (size_t)c * (dim + 1);
        for (uint64_t d = bounds[c]; d < bounds[c + 1]; ++d)
            for (uint64_t j = row_ptr[d]; j < row_ptr[d + 1]; ++j) {
                uint32_t t = word_term(words[j]);
                uint64_t p = pos[t]++;
                out.doc[p] = (uint32_t)d;
                out.val[p] = word_half(words[j]);
            }
    });
}

// ----------------------------------------------------------------- build

uint32_t HostIndex::max_blocks_per_list() const {
    uint32_t mx = 0;
    for (uint32_t t = 0; t < dim; ++t) mx = std::max(mx, list_off[t + 1] - list_off[t]);
    return mx;
}

namespace {

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the build's own stream for centroid sampling.
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
};

struct TermOut {
    std::vector<uint32_t> post_len;   // per block
    std::vector<uint32_t> postings;
    std::vector<uint32_t> sum_len;    // per block
    std::vector<uint16_t> sum_term;
    std::vector<uint8_t> sum_code;
    std::vector<float> m, delta;
    std::vector<uint32_t> centroid;
};

struct Scratch {
    std::vector<double> acc;                    // per centroid
    std::vector<uint32_t> ctab_start, ctab_cnt; // per term: centroid postings
    std::vector<uint32_t> ctab_touched;
    std::vector<uint32_t> c_k;                  // centroid postings: centroid index
    std::vector<float> c_v;                     //                     value
    std::vector<uint16_t> phi;                  // per term, fp16 bits of the max
    std::vector<uint32_t> touched;
    std::vector<std::pair<uint64_t, uint32_t>> ent;
    std::vector<uint32_t> perm, assign, count, order;
    std::vector<std::pair<uint64_t, uint32_t>> col;
    explicit Scratch(uint32_t dim) : ctab_start(dim, 0), ctab_cnt(dim, 0), phi(dim, 0) {}
};

// u8 quantization on the 2^-14 grid: m = min rounded down, sub-interval
// size = (max - m) / 256 rounded up, code = floor((v - m) / size) clamped to
// 255.  Exact integer arithmetic on multiples of 2^-24.
void quantize_block(const uint16_t* vals, size_t n, float& m_out, float& d_out, uint8_t* codes) {
    uint64_t vmin = UINT64_MAX, vmax = 0;
    for (size_t i = 0; i < n; ++i) {
        uint64_t v = half_units24(vals[i]);
        vmin = std::min(vmin, v);
        vmax = std::max(vmax, v);
    }
    const uint64_t grid = 1ull << (24 - kGridBits);
    uint64_t m_u = (vmin / grid) * grid;
    uint64_t span = vmax - m_u;
    uint64_t d_u = ((span + 256 * grid - 1) / (256 * grid)) * grid;
    for (size_t i = 0; i < n; ++i) {
        uint64_t c = d_u ? (half_units24(vals[i]) - m_u) / d_u : 0;
        codes[i] = (uint8_t)std::min<uint64_t>(c, 255);
    }
    m_out = (float)std::ldexp((double)m_u, -24);
    d_out = (float)std::ldexp((double)d_u, -24);
}

}  // namespace

// Entries kept of a column of n_full nonzeros (Set alpha-MSS, Section 3.4):
// the fixed cap lambda, and with alpha > 0 also at most ceil(alpha * n_full)
// (the proportional form), at least 1.
uint64_t list_cap(uint64_t n_full, uint32_t lambda, double alpha) {
    uint64_t cap = lambda;
    if (alpha > 0.0) {
        const double c = std::ceil(alpha * (double)n_full);
        const uint64_t pc = c < 1.0 ? 1 : (uint64_t)c;
        if (pc < cap) cap = pc;
    }
    return cap;
}

namespace {

void build_term(uint32_t t, const HostCSC& csc, const uint64_t* row_ptr, const uint32_t* words,
                const seismic_build_params& p, uint32_t dim, Scratch& S, TermOut& out) {
    const uint64_t a = csc.off[t], b = csc.off[t + 1];
    const uint64_t n_full = b - a;
    if (n_full == 0) return;
    // Set alpha-MSS: keep the cap largest values of the column (value desc,
    // doc id asc); the kept list is stored doc-ascending.
    const uint64_t cap = list_cap(n_full, p.lambda, p.alpha);
    std::vector<uint32_t> list;
    if (n_full <= cap) {
        list.assign(csc.doc.begin() + a, csc.doc.begin() + b);
    } else {
        S.col.resize(n_full);
        for (uint64_t i = 0; i < n_full; ++i)  // key: larger value first, then smaller id
            S.col[i] = {~half_units24(csc.val[a + i]), csc.doc[a + i]};
        std::nth_element(S.col.begin(), S.col.begin() + (cap - 1), S.col.end());
        // nth_element leaves the smallest cap keys (by pair order) in front
        list.resize(cap);
        for (uint64_t i = 0; i < cap; ++i) list[i] = S.col[i].second;
        std::sort(list.begin(), list.end());
    }
    const uint64_t n = list.size();
    uint64_t nb = ((uint64_t)p.beta * n + p.lambda - 1) / p.lambda;
    if (nb < 1) nb = 1;
    if (nb > n) nb = n;
    // Shallow K-means (Section 4.1.2): nb distinct members sampled uniformly
    // as centroids; each document joins argmax_k <u, mu_k> (lowest k on ties).
    S.perm.resize(n);
    std::iota(S.perm.begin(), S.perm.end(), 0u);
    SplitMix64 rng{p.seed ^ (0xD1B54A32D192ED03ull * ((uint64_t)t + 1))};
    for (uint64_t i = 0; i < nb; ++i) std::swap(S.perm[i], S.perm[i + rng.below(n - i)]);
    S.assign.assign(n, 0);
    if (nb > 1) {
        // inverted index of the centroids: term -> (centroid, value)
        S.ctab_touched.clear();
        for (uint64_t k = 0; k < nb; ++k) {
            uint32_t c = list[S.perm[k]];
            for (uint64_t j = row_ptr[c]; j < row_ptr[c + 1]; ++j) {
                uint32_t tt = word_term(words[j]);
                if (S.ctab_cnt[tt]++ == 0) S.ctab_touched.push_back(tt);
            }
        }
        uint32_t run = 0;
        for (uint32_t tt : S.ctab_touched) { S.ctab_start[tt] = run; run += S.ctab_cnt[tt]; S.ctab_cnt[tt] = 0; }
        S.c_k.resize(run);
        S.c_v.resize(run);
        for (uint64_t k = 0; k < nb; ++k) {
            uint32_t c = list[S.perm[k]];
            for (uint64_t j = row_ptr[c]; j < row_ptr[c + 1]; ++j) {
                uint32_t tt = word_term(words[j]);
                uint32_t pos = S.ctab_start[tt] + S.ctab_cnt[tt]++;
                S.c_k[pos] = (uint32_t)k;
                S.c_v[pos] = half_to_float(word_half(words[j]));
            }
        }
        S.acc.assign(nb, 0.0);
        for (uint64_t i = 0; i < n; ++i) {
            uint32_t d = list[i];
            for (uint64_t j = row_ptr[d]; j < row_ptr[d + 1]; ++j) {
                uint32_t tt = word_term(words[j]);
                uint32_t cnt = S.ctab_cnt[tt];
                if (!cnt) continue;
                double v = (double)half_to_float(word_half(words[j]));
                const uint32_t s0 = S.ctab_start[tt];
                for (uint32_t e = 0; e < cnt; ++e) S.acc[S.c_k[s0 + e]] += v * (double)S.c_v[s0 + e];
            }
            uint32_t best = 0;
            double bv = S.acc[0];
            for (uint64_t k = 1; k < nb; ++k)
                if (S.acc[k] > bv) { bv = S.acc[k]; best = (uint32_t)k; }
            S.assign[i] = best;
            std::fill(S.acc.begin(), S.acc.end(), 0.0);
        }
        for (uint32_t tt : S.ctab_touched) S.ctab_cnt[tt] = 0;
    }
    // blocks in centroid order, empty clusters dropped, docs ascending
    S.count.assign(nb + 1, 0);
    for (uint64_t i = 0; i < n; ++i) S.count[S.assign[i] + 1]++;
    for (uint64_t k = 0; k < nb; ++k) S.count[k + 1] += S.count[k];
    S.order.resize(n);
    {
        std::vector<uint32_t> pos(S.count.begin(), S.count.end() - 1);
        for (uint64_t i = 0; i < n; ++i) S.order[pos[S.assign[i]]++] = list[i];
    }
    for (uint64_t k = 0; k < nb; ++k) {
        uint32_t c0 = S.count[k], c1 = S.count[k + 1];
        if (c1 == c0) continue;
        out.post_len.push_back(c1 - c0);
        out.postings.insert(out.postings.end(), S.order.begin() + c0, S.order.begin() + c1);
        out.centroid.push_back(list[S.perm[k]]);
        // phi(B)_i = max over the block's documents (full vectors)
        S.touched.clear();
        for (uint32_t q = c0; q < c1; ++q) {
            uint32_t d = S.order[q];
            for (uint64_t j = row_ptr[d]; j < row_ptr[d + 1]; ++j) {
                uint32_t tt = word_term(words[j]);
                uint16_t h = word_half(words[j]);
                if (S.phi[tt] == 0) S.touched.push_back(tt);
                if (h > S.phi[tt]) S.phi[tt] = h;  // positive fp16: bit order is value order
            }
        }
        // gamma-MSS of phi: value desc (ties: term asc), shortest prefix with
        // mass >= gamma * total (fp64 sums, exact for fp16 values)
        S.ent.clear();
        double total = 0.0;
        for (uint32_t tt : S.touched) {
            uint64_t u = half_units24(S.phi[tt]);
            S.ent.push_back({~u, tt});
            total += std::ldexp((double)u, -24);
        }
        // The kept prefix is found by selection, not a full sort: halve the
        // candidate range [lo, hi) around its rank-median (nth_element) while
        // tracking the mass of the best elements known to be kept; the sums
        // are exact, so the boundary equals the one of the sorted scan.
        const double need = p.gamma * total;
        size_t lo = 0, hi = S.ent.size();
        double before = 0.0;  // mass of ent[0, lo): all kept
        while (hi - lo > 32) {
            const size_t mid = lo + (hi - lo) / 2;
            std::nth_element(S.ent.begin() + lo, S.ent.begin() + mid, S.ent.begin() + hi);
            double m = 0.0;
            for (size_t i = lo; i <= mid; ++i) m += std::ldexp((double)(~S.ent[i].first), -24);
            if (before + m >= need) {
                hi = mid + 1;
            } else {
                before += m;
                lo = mid + 1;
            }
        }
        std::sort(S.ent.begin() + lo, S.ent.begin() + hi);
        double cum = before;
        size_t keep = lo;
        while (keep < S.ent.size()) {
            cum += std::ldexp((double)(~S.ent[keep].first), -24);
            ++keep;
            if (cum >= need) break;
        }
        std::vector<std::pair<uint32_t, uint16_t>> kept(keep);
        for (size_t i = 0; i < keep; ++i) kept[i] = {S.ent[i].second, S.phi[S.ent[i].second]};
        for (uint32_t tt : S.touched) S.phi[tt] = 0;
        std::sort(kept.begin(), kept.end());
        std::vector<uint16_t> vals(keep);
        std::vector<uint8_t> codes(keep);
        for (size_t i = 0; i < keep; ++i) vals[i] = kept[i].second;
        float m, dl;
        quantize_block(vals.data(), keep, m, dl, codes.data());
        out.m.push_back(m);
        out.delta.push_back(dl);
        out.sum_len.push_back((uint32_t)keep);
        for (size_t i = 0; i < keep; ++i) {
            out.sum_term.push_back((uint16_t)kept[i].first);
            out.sum_code.push_back(codes[i]);
        }
    }
}

}  // namespace

int build_host_index(const seismic_csr* docs, const seismic_build_params* p, HostIndex& H) {
    if (!p) return fail(SEISMIC_EINVAL, "build: null params");
    if (p->lambda < 1) return fail(SEISMIC_EINVAL, "build: lambda must be >= 1");
    if (p->beta < 1) return fail(SEISMIC_EINVAL, "build: beta must be >= 1");
    if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return fail(SEISMIC_EINVAL, "build: gamma must be in (0, 1]");
    if (!(p->alpha >= 0.0 && p->alpha <= 1.0)) return fail(SEISMIC_EINVAL, "build: alpha must be in [0, 1]");
    int rc = validate_csr_host(docs, 65536, "build: docs");
    if (rc) return rc;
    if (docs->n_rows >= 0xFFFFFFFFull) return fail(SEISMIC_EINVAL, "build: more than 2^32-1 documents");
    const int nthreads = resolve_threads(p->n_threads);
    const uint32_t dim = docs->dim;
    try {
        H = HostIndex();
        H.dim = dim;
        H.n_docs = docs->n_rows;
        H.lambda = p->lambda;
        H.beta = p->beta;
        H.gamma = p->gamma;
        H.seed = p->seed;
        H.alpha = p->alpha;
        H.row_ptr.assign(docs->row_ptr, docs->row_ptr + docs->n_rows + 1);
        H.words.assign(docs->words, docs->words + docs->nnz);
        auto t_start = std::chrono::steady_clock::now();
        auto elapsed = [&]() {
            return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        };
        HostCSC csc;
        build_csc(H.row_ptr.data(), H.words.data(), H.n_docs, dim, nthreads, csc);
        if (p->verbose) std::fprintf(stderr, "build: inverted lists done (%.1f s, %d threads)\n", elapsed(), nthreads);
        std::vector<TermOut> outs(dim);
        // largest lists first for load balance
        std::vector<uint32_t> terms(dim);
        std::iota(terms.begin(), terms.end(), 0u);
        std::sort(terms.begin(), terms.end(), [&](uint32_t x, uint32_t y) {
            uint64_t nx = std::min<uint64_t>(csc.off[x + 1] - csc.off[x], list_cap(csc.off[x + 1] - csc.off[x], p->lambda, p->alpha));
            uint64_t ny = std::min<uint64_t>(csc.off[y + 1] - csc.off[y], list_cap(csc.off[y + 1] - csc.off[y], p->lambda, p->alpha));
            return nx != ny ? nx > ny : x < y;
        });
        std::vector<std::unique_ptr<Scratch>> scratch(nthreads);
        for (auto& s : scratch) s.reset(new Scratch(dim));
        uint64_t total_work = 0;
        for (uint32_t t = 0; t < dim; ++t) total_work += std::min<uint64_t>(csc.off[t + 1] - csc.off[t], list_cap(csc.off[t + 1] - csc.off[t], p->lambda, p->alpha));
        std::atomic<uint64_t> done_work{0};
        std::atomic<int> reported{0};
        parallel_for(dim, nthreads, 1, [&](int64_t i, int tid) {
            uint32_t t = terms[i];
            build_term(t, csc, H.row_ptr.data(), H.words.data(), *p, dim, *scratch[tid], outs[t]);
            if (p->verbose && total_work) {
                uint64_t w = std::min<uint64_t>(csc.off[t + 1] - csc.off[t], list_cap(csc.off[t + 1] - csc.off[t], p->lambda, p->alpha));
                uint64_t d = done_work.fetch_add(w) + w;
                int pct = (int)(100 * d / total_work);
                int prev = reported.load();
                while (pct >= prev + 10 && !reported.compare_exchange_weak(prev, pct - pct % 10)) {}
                if (pct >= prev + 10) std::fprintf(stderr, "build: lists %d%% (%.1f s)\n", pct - pct % 10, elapsed());
            }
        });
        csc = HostCSC();
        if (p->verbose) std::fprintf(stderr, "build: blocks and summaries done (%.1f s)\n", elapsed());
        // concatenate in term order
        uint64_t nb = 0, np = 0, ns = 0;
        for (auto& o : outs) { nb += o.m.size(); np += o.postings.size(); ns += o.sum_term.size(); }
        if (np >= 0xFFFFFFFFull || nb >= 0xFFFFFFFFull) return fail(SEISMIC_ENOMEM, "build: index exceeds 32-bit offsets");
        H.list_off.resize((size_t)dim + 1);
        H.blk_post_off.resize(nb + 1);
        H.blk_sum_off.resize(nb + 1);
        H.blk_m.resize(nb);
        H.blk_delta.resize(nb);
        H.blk_centroid.resize(nb);
        H.postings.resize(np);
        H.sum_term.resize(ns);
        H.sum_code.resize(ns);
        uint64_t b = 0, pp = 0, ss = 0;
        for (uint32_t t = 0; t < dim; ++t) {
            H.list_off[t] = (uint32_t)b;
            TermOut& o = outs[t];
            for (size_t j = 0; j < o.m.size(); ++j) {
                H.blk_post_off[b] = (uint32_t)pp;
                H.blk_sum_off[b] = ss;
                H.blk_m[b] = o.m[j];
                H.blk_delta[b] = o.delta[j];
                H.blk_centroid[b] = o.centroid[j];
                pp += o.post_len[j];
                ss += o.sum_len[j];
                ++b;
            }
            std::copy(o.postings.begin(), o.postings.end(), H.postings.begin() + (pp - o.postings.size()));
            std::copy(o.sum_term.begin(), o.sum_term.end(), H.sum_term.begin() + (ss - o.sum_term.size()));
            std::copy(o.sum_code.begin(), o.sum_code.end(), H.sum_code.begin() + (ss - o.sum_code.size()));
            o = TermOut();
        }
        H.list_off[dim] = (uint32_t)b;
        H.blk_post_off[nb] = (uint32_t)pp;
        H.blk_sum_off[nb] = ss;
    } catch (const std::bad_alloc&) {
        return fail(SEISMIC_ENOMEM, "build: host allocation failed");
    }
    return SEISMIC_OK;
}

// ------------------------------------------------------------- serialize

static uint64_t al64(uint64_t x) { return (x + 63) & ~63ull; }

struct SectionView {
    const void* p;
    uint64_t bytes;
};

static void sections_of(const HostIndex& h, SectionView s[11]) {
    s[0] = {h.row_ptr.data(), 8 * h.row_ptr.size()};
    s[1] = {h.words.data(), 4 * h.words.size()};
    s[2] = {h.list_off.data(), 4 * h.list_off.size()};
    s[3] = {h.blk_post_off.data(), 4 * h.blk_post_off.size()};
    s[4] = {h.blk_sum_off.data(), 8 * h.blk_sum_off.size()};
    s[5] = {h.blk_m.data(), 4 * h.blk_m.size()};
    s[6] = {h.blk_delta.data(), 4 * h.blk_delta.size()};
    s[7] = {h.blk_centroid.data(), 4 * h.blk_centroid.size()};
    s[8] = {h.postings.data(), 4 * h.postings.size()};
    s[9] = {h.sum_term.data(), 2 * h.sum_term.size()};
    s[10] = {h.sum_code.data(), h.sum_code.size()};
}

uint64_t serialized_size(const HostIndex& h) {
    SectionView s[11];
    sections_of(h, s);
    uint64_t off = kHeaderBytes;
    for (auto& v : s) off = al64(off) + v.bytes;
    return al64(off);
}

void serialize(const HostIndex& h, uint8_t* buf) {
    uint8_t head[kHeaderBytes];
    std::memset(head, 0, sizeof(head));
    std::memcpy(head, "SEISMIC", 8);
    uint32_t u32;
    uint64_t u64;
    u32 = kFormatVersion; std::memcpy(head + 8, &u32, 4);
    std::memcpy(head + 12, &h.dim, 4);
    std::memcpy(head + 16, &h.n_docs, 8);
    u64 = h.nnz(); std::memcpy(head + 24, &u64, 8);
    u64 = h.n_blocks(); std::memcpy(head + 32, &u64, 8);
    u64 = h.postings.size(); std::memcpy(head + 40, &u64, 8);
    u64 = h.sum_term.size(); std::memcpy(head + 48, &u64, 8);
    std::memcpy(head + 56, &h.lambda, 4);
    std::memcpy(head + 60, &h.beta, 4);
    std::memcpy(head + 64, &h.gamma, 8);
    std::memcpy(head + 72, &h.seed, 8);
    u32 = kGridBits; std::memcpy(head + 80, &u32, 4);
    std::memcpy(head + 88, &h.alpha, 8);
    std::memcpy(buf, head, kHeaderBytes);
    SectionView s[11];
    sections_of(h, s);
    uint64_t off = kHeaderBytes;
    for (auto& v : s) {
        uint64_t a = al64(off);
        if (a > off) std::memset(buf + off, 0, a - off);
        if (v.bytes) std::memcpy(buf + a, v.p, v.bytes);
        off = a + v.bytes;
    }
    uint64_t end = al64(off);
    if (end > off) std::memset(buf + off, 0, end - off);
}

int deserialize(const uint8_t* buf, uint64_t size, HostIndex& h) {
    if (size < kHeaderBytes || std::memcmp(buf, "SEISMIC", 8) != 0)
        return fail(SEISMIC_EFORMAT, "index: bad magic");
    uint32_t version, grid;
    uint64_t nnz, nb, np, ns;
    std::memcpy(&version, buf + 8, 4);
    if (version != kFormatVersion) return fail(SEISMIC_EFORMAT, "index: unsupported version %u", version);
    std::memcpy(&h.dim, buf + 12, 4);
    std::memcpy(&h.n_docs, buf + 16, 8);
    std::memcpy(&nnz, buf + 24, 8);
    std::memcpy(&nb, buf + 32, 8);
    std::memcpy(&np, buf + 40, 8);
    std::memcpy(&ns, buf + 48, 8);
    std::memcpy(&h.lambda, buf + 56, 4);
    std::memcpy(&h.beta, buf + 60, 4);
    std::memcpy(&h.gamma, buf + 64, 8);
    std::memcpy(&h.seed, buf + 72, 8);
    std::memcpy(&grid, buf + 80, 4);
    std::memcpy(&h.alpha, buf + 88, 8);
    if (!(h.alpha >= 0.0 && h.alpha <= 1.0)) return fail(SEISMIC_EFORMAT, "index: alpha out of range");
    if (grid != kGridBits) return fail(SEISMIC_EFORMAT, "index: unsupported quantization grid");
    if (h.dim < 1 || h.dim > 65536 || h.n_docs >= 0xFFFFFFFFull || np >= 0xFFFFFFFFull || nb >= 0xFFFFFFFFull)
        return fail(SEISMIC_EFORMAT, "index: header out of range");
    uint64_t sizes[11] = {8 * (h.n_docs + 1), 4 * nnz, 4 * ((uint64_t)h.dim + 1), 4 * (nb + 1), 8 * (nb + 1),
                          4 * nb, 4 * nb, 4 * nb, 4 * np, 2 * ns, ns};
    uint64_t off = kHeaderBytes;
    uint64_t starts[11];
    for (int i = 0; i < 11; ++i) {
        off = al64(off);
        if (sizes[i] > size || off > size - sizes[i]) return fail(SEISMIC_EFORMAT, "index: truncated (section %d)", i);
        starts[i] = off;
        off += sizes[i];
    }
    try {
        auto take = [&](auto& vec, int i) {
            using T = typename std::decay_t<decltype(vec)>::value_type;
            vec.resize(sizes[i] / sizeof(T));
            if (sizes[i]) std::memcpy(vec.data(), buf + starts[i], sizes[i]);
        };
        take(h.row_ptr, 0); take(h.words, 1); take(h.list_off, 2); take(h.blk_post_off, 3);
        take(h.blk_sum_off, 4); take(h.blk_m, 5); take(h.blk_delta, 6); take(h.blk_centroid, 7);
        take(h.postings, 8); take(h.sum_term, 9); take(h.sum_code, 10);
    } catch (const std::bad_alloc&) {
        return fail(SEISMIC_ENOMEM, "index: host allocation failed");
    }
    // structural validation: everything the kernels index with must be in range
    if (h.row_ptr[0] != 0 || h.row_ptr[h.n_docs] != nnz) return fail(SEISMIC_EFORMAT, "index: bad row_ptr");
    for (uint64_t i = 0; i < h.n_docs; ++i)
        if (h.row_ptr[i] > h.row_ptr[i + 1]) return fail(SEISMIC_EFORMAT, "index: row_ptr not monotone");
    if (h.list_off[0] != 0 || h.list_off[h.dim] != nb) return fail(SEISMIC_EFORMAT, "index: bad list offsets");
    for (uint32_t t = 0; t < h.dim; ++t)
        if (h.list_off[t] > h.list_off[t + 1]) return fail(SEISMIC_EFORMAT, "index: list offsets not monotone");
    if (h.blk_post_off[0] != 0 || h.blk_post_off[nb] != np || h.blk_sum_off[0] != 0 || h.blk_sum_off[nb] != ns)
        return fail(SEISMIC_EFORMAT, "index: bad block offsets");
    for (uint64_t b = 0; b < nb; ++b)
        if (h.blk_post_off[b] > h.blk_post_off[b + 1] || h.blk_sum_off[b] > h.blk_sum_off[b + 1])
            return fail(SEISMIC_EFORMAT, "index: block offsets not monotone");
    for (uint64_t b = 0; b < nb; ++b)
        if (!(std::isfinite(h.blk_m[b]) && h.blk_m[b] >= 0.0f && std::isfinite(h.blk_delta[b]) && h.blk_delta[b] >= 0.0f))
            return fail(SEISMIC_EFORMAT, "index: block %llu has a bad quantization range", (unsigned long long)b);
    for (uint64_t i = 0; i < np; ++i)
        if (h.postings[i] >= h.n_docs) return fail(SEISMIC_EFORMAT, "index: posting out of range");
    for (uint64_t i = 0; i < ns; ++i)
        if (h.sum_term[i] >= h.dim) return fail(SEISMIC_EFORMAT, "index: summary term out of range");
    for (uint64_t i = 0; i < nnz; ++i)
        if (word_term(h.words[i]) >= h.dim) return fail(SEISMIC_EFORMAT, "index: forward term out of range");
    for (uint64_t d = 0; d < h.n_docs; ++d)
        if (h.row_ptr[d + 1] - h.row_ptr[d] > 65536) return fail(SEISMIC_EFORMAT, "index: row too long");
    return SEISMIC_OK;
}

}  // namespace seismic

using namespace seismic;

extern "C" {

const char* seismic_last_error(void) { return last_error_cstr(); }

int seismic_build_index(const seismic_csr* docs, const seismic_build_params* params, seismic_index** out) {
    if (!out) return fail(SEISMIC_EINVAL, "build: null output");
    *out = nullptr;
    seismic_index* ix = new (std::nothrow) seismic_index();
    if (!ix) return fail(SEISMIC_ENOMEM, "build: host allocation failed");
    int rc = build_host_index(docs, params, ix->h);
    if (rc) { delete ix; return rc; }
    *out = ix;
    return SEISMIC_OK;
}

int seismic_index_serialized_size(const seismic_index* index, uint64_t* bytes) {
    if (!index || !bytes) return fail(SEISMIC_EINVAL, "serialized_size: null argument");
    const HostIndex& h = index->h;
    SectionView sv[11];
    sections_of(h, sv);
    if (index->device_only) {  // the device-resident sections, by size
        sv[0].bytes = 8 * (h.n_docs + 1);
        sv[1].bytes = 4 * index->dev_nnz;
        sv[8].bytes = 4 * index->dev_postings;
        sv[9].bytes = 2 * index->dev_sums;
        sv[10].bytes = index->dev_sums;
    }
    uint64_t off = kHeaderBytes;
    for (auto& v : sv) off = al64(off) + v.bytes;
    *bytes = al64(off);
    return SEISMIC_OK;
}

int seismic_index_serialize(const seismic_index* index, void* buf, uint64_t bytes) {
    if (!index || !buf) return fail(SEISMIC_EINVAL, "serialize: null argument");
    HostIndex tmp;
    const HostIndex* h = nullptr;
    int rc = full_host_index(index, tmp, &h);
    if (rc) return rc;
    if (bytes < serialized_size(*h)) return fail(SEISMIC_EINVAL, "serialize: buffer too small");
    serialize(*h, (uint8_t*)buf);
    return SEISMIC_OK;
}

int seismic_index_save(const seismic_index* index, const char* path) {
    if (!index || !path) return fail(SEISMIC_EINVAL, "save: null argument");
    HostIndex tmp;
    const HostIndex* h = nullptr;
    int rc = full_host_index(index, tmp, &h);
    if (rc) return rc;
    uint64_t n = serialized_size(*h);
    std::vector<uint8_t> buf;
    try { buf.resize(n); } catch (const std::bad_alloc&) { return fail(SEISMIC_ENOMEM, "save: host allocation failed"); }
    serialize(*h, buf.data());
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SEISMIC_EIO, "save: cannot open %s", path);
    size_t w = std::fwrite(buf.data(), 1, n, f);
    int cl = std::fclose(f);
    if (w != n || cl != 0) return fail(SEISMIC_EIO, "save: write to %s failed", path);
    return SEISMIC_OK;
}

int seismic_index_load(const char* path, seismic_index** out) {
    if (!path || !out) return fail(SEISMIC_EINVAL, "load: null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SEISMIC_EIO, "load: cannot open %s", path);
    std::fseek(f, 0, SEEK_END);
    long sz = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    if (sz < 0) { std::fclose(f); return fail(SEISMIC_EIO, "load: cannot size %s", path); }
    std::vector<uint8_t> buf;
    try { buf.resize((size_t)sz); } catch (const std::bad_alloc&) { std::fclose(f); return fail(SEISMIC_ENOMEM, "load: host allocation failed"); }
    size_t r = std::fread(buf.data(), 1, (size_t)sz, f);
    std::fclose(f);
    if (r != (size_t)sz) return fail(SEISMIC_EIO, "load: short read of %s", path);
    seismic_index* ix = new (std::nothrow) seismic_index();
    if (!ix) return fail(SEISMIC_ENOMEM, "load: host allocation failed");
    int rc = deserialize(buf.data(), buf.size(), ix->h);
    if (rc) { delete ix; return rc; }
    *out = ix;
    return SEISMIC_OK;
}

int seismic_index_info(const seismic_index* index, uint64_t out[10]) {
    if (!index || !out) return fail(SEISMIC_EINVAL, "info: null argument");
    const HostIndex& h = index->h;
    out[0] = h.dim; out[1] = h.n_docs; out[2] = index->nnz(); out[3] = h.n_blocks();
    out[4] = index->device_only ? index->dev_postings : h.postings.size();
    out[5] = index->device_only ? index->dev_sums : h.sum_term.size();
    out[6] = h.lambda; out[7] = h.beta;
    out[8] = h.max_blocks_per_list();
    out[9] = device_index_layout(index->dev);
    return SEISMIC_OK;
}

void seismic_index_free(seismic_index* index) {
    if (!index) return;
    if (index->dev) device_index_free(index->dev);
    delete index;
}

}  // extern "C"
