// Algorithm 2 ("Query processing with Seismic", Section 4.5) with the
// kappa-NN refinement disabled.  One workgroup of NT threads answers one
// query at a time; a persistent grid pulls query indices from a device
// counter.
//
//   1. ingest: the query becomes a dense u8 slot table over all terms in LDS
//      (slot 0 = absent) plus an fp64 value per slot, value[0] = 0, so every
//      lookup is two LDS reads and no branch; queries with more than 255
//      distinct terms use a membership bitmap with prefix counts instead.
//      The cut keeps the query_cut largest entries (value desc, term asc);
//   2. per cut list, in cut order:
//      a. summary scores r_j = <q, S_j> of every block: the list's summary
//         entries are one contiguous run, streamed by the whole workgroup in
//         16-byte groups of 8 entries; per block, sum(q) and sum(q * code)
//         are gathered in LDS fp64 and r_j = m_j * sum(q) + delta_j *
//         sum(q * code) (exact for values in [2^-6, 2^6]: m and delta sit on
//         the 2^-14 grid, so every term is a multiple of 2^-30 below 2^23);
//      b. blocks that can never be evaluated in this list (full heap and
//         r * heap_factor < heap.min, which only grows) are dropped, the rest
//         sorted in LDS by (r desc, block asc) with a bitonic network;
//      c. traversal in that order: up to W consecutive blocks (at most NT
//         documents) are gathered at once - a thread per document fetches
//         its posting and row offsets, then groups of 4 lanes stream whole
//         rows as 16-byte loads and accumulate exact products in fp64 - and
//         the blocks are then replayed one by one: a block is evaluated
//         unless the heap is full and r * heap_factor < heap.min, which ends
//         the list; an evaluated block's documents are folded into the LDS
//         top-k.  Replaying in order keeps every decision identical to the
//         sequential algorithm; blocks gathered past a stop are wasted work.
//      With a learned probe, a list whose traversal starts with a full heap
//      instead evaluates exactly the blocks whose probe logit (computed once,
//      from the heap minimum at the list's start) is >= tau: b. keeps those
//      blocks, nothing is sorted and c. makes no prune decisions.
#include "device_common.h"
#include "probe.h"
#include "search_kernels.h"

namespace seismic_dev {

constexpr uint32_t kUnroll = 2;       // 16-byte row loads in flight per document and lane
constexpr uint32_t kLanesPerDoc = 4;  // lanes sharing one row
constexpr uint32_t kDocsPerGroup = 2; // rows a group of lanes streams at a time
constexpr uint32_t kSumUnroll = 2;    // summary groups in flight per thread
constexpr uint32_t kMaxSlots = 255;   // distinct query terms served by the u8 slot table

template <int NT>
struct SearchLds {
    uint8_t* region;  // all-zero between queries: u8 slot table, or bitmap + prefix + values
    uint32_t region_bytes;
    double* qv;       // [256] value by slot (u8 mode), qv[0] = 0
    QTable bq;        // bitmap mode, aliased on region
    uint16_t* cut;    // [kMaxQ]
    uint32_t* soff;   // [P + 1] summary offsets of the list's blocks, list-relative
    float* r;         // [P] surviving blocks' summary scores (sorted in place)
    uint16_t* ord;    // [P] their block index within the list
    uint32_t* wp0;    // [kMaxW] window: first posting of each block
    uint32_t* wlen;   // [kMaxW]  documents of each block
    uint32_t* wst;    // [kMaxW + 1] prefix of wlen
    uint32_t* scratch;
    uint32_t* misc;
    // union region
    uint16_t* q_term;  // ingest [kMaxQ]
    uint16_t* q_half;  // ingest [kMaxQ]
    double* A;         // summary phase [P]
    double* B;         // summary phase [P]
    uint32_t* cdoc;    // gather phase [NT]
    uint64_t* crs;     // [NT]
    uint32_t* clen;    // [NT] row lengths
    double* cacc;      // [NT]
    uint8_t* cslot;    // [NT]
    // wide schedule traversal only (carved past the common layout): the
    // speculated blocks of the current list by sorted position
    uint32_t* wfirst;  // [kWideMaxDepth] first evaluation item
    uint32_t* wdocs;   // [kWideMaxDepth] documents
    uint64_t* wnnz;    // [kWideMaxDepth] nonzeros
    // and every cut list's header, loaded at once
    uint32_t* wl_b0;   // [kWideMaxCut] first block
    uint32_t* wl_nb;   // [kWideMaxCut] blocks
    uint32_t* wl_D;    // [kWideMaxCut] speculated blocks
    uint64_t* wl_S0;   // [kWideMaxCut] summary entries [S0, S1)
    uint64_t* wl_S1;   // [kWideMaxCut]
    int64_t* wl_cb;    // [kWideMaxCut] copy_bias of the list
};

__host__ __device__ inline uint32_t r16u(uint64_t x) { return (uint32_t)((x + 15) & ~uint64_t(15)); }

__host__ __device__ inline uint32_t region_bytes_for(uint32_t dim) {
    const uint32_t nw = (dim + 63) / 64;
    const uint32_t bitmap = r16u(8ull * nw) + r16u(2ull * nw) + r16u(4ull * kMaxQ);
    const uint32_t table = r16u(dim);
    return bitmap > table ? bitmap : table;
}

template <int NT>
__host__ __device__ inline size_t union_bytes(uint32_t P) {
    size_t ingest = 2 * 2 * (size_t)kMaxQ + 32;
    size_t summ = 2 * 8 * (size_t)P + 32;
    size_t gath = (size_t)NT * (8 + 8 + 4 + 4 + 1) + 6 * 16;
    size_t m = ingest > summ ? ingest : summ;
    return m > gath ? m : gath;
}

// Returns the end of the layout (search_smem_bytes past base).
template <int NT>
__device__ inline uint8_t* carve_lds(uint8_t* base, uint32_t dim, uint32_t P, uint32_t k, SearchLds<NT>& L,
                                     TopK<NT>& top) {
    const uint32_t nw = (dim + 63) / 64;
    uint8_t* p = base;
    L.region_bytes = region_bytes_for(dim);
    L.region = carve(p, L.region_bytes);
    {
        uint8_t* b = L.region;
        L.bq.bits = (uint64_t*)carve(b, 8ull * nw);
        L.bq.pref = (uint16_t*)carve(b, 2ull * nw);
        L.bq.val = (float*)carve(b, 4ull * kMaxQ);
    }
    L.qv = (double*)carve(p, 8ull * 256);
    L.cut = (uint16_t*)carve(p, 2ull * kMaxQ);
    L.soff = (uint32_t*)carve(p, 4ull * (P + 1));
    L.r = (float*)carve(p, 4ull * P);
    L.ord = (uint16_t*)carve(p, 2ull * P);
    L.wp0 = (uint32_t*)carve(p, 4ull * kMaxW);
    L.wlen = (uint32_t*)carve(p, 4ull * kMaxW);
    L.wst = (uint32_t*)carve(p, 4ull * (kMaxW + 1));
    L.scratch = (uint32_t*)carve(p, 4ull * (NT / kWave + 8));
    L.misc = (uint32_t*)carve(p, 4ull * 16);
    top.s0 = (float*)carve(p, 4ull * k);
    top.s1 = (float*)carve(p, 4ull * k);
    top.i0 = (uint32_t*)carve(p, 4ull * k);
    top.i1 = (uint32_t*)carve(p, 4ull * k);
    top.cs = (float*)carve(p, 4ull * NT);
    top.cid = (uint32_t*)carve(p, 4ull * NT);
    top.scratch = L.scratch;
    top.which = 0;
    top.hn = 0;
    top.k = k;
    uint8_t* u = p;
    uint8_t* q = u;
    L.q_term = (uint16_t*)carve(q, 2ull * kMaxQ);
    L.q_half = (uint16_t*)carve(q, 2ull * kMaxQ);
    q = u;
    L.A = (double*)carve(q, 8ull * P);
    L.B = (double*)carve(q, 8ull * P);
    q = u;
    L.cacc = (double*)carve(q, 8ull * NT);
    L.crs = (uint64_t*)carve(q, 8ull * NT);
    L.cdoc = (uint32_t*)carve(q, 4ull * NT);
    L.clen = (uint32_t*)carve(q, 4ull * NT);
    L.cslot = (uint8_t*)carve(q, 1ull * NT);
    return u + union_bytes<NT>(P);
}

// The wide evaluation pass's layout: what one item needs (lookup region,
// slot values, a one-block window, top-k, ingest and gather scratch) and
// none of the list traversal's arrays (cut, block offsets, scores, order,
// summary sums).  The merge candidates live in the row-start array, which
// is dead once the item's documents are scored, so at k <= kWideMaxK four
// workgroups fit a CU.
__device__ inline void carve_lds_eval(uint8_t* base, uint32_t dim, uint32_t k, SearchLds<kWideChunk>& L,
                                      TopK<kWideChunk>& top) {
    constexpr int NT = kWideChunk;
    const uint32_t nw = (dim + 63) / 64;
    uint8_t* p = base;
    L.region_bytes = region_bytes_for(dim);
    L.region = carve(p, L.region_bytes);
    {
        uint8_t* b = L.region;
        L.bq.bits = (uint64_t*)carve(b, 8ull * nw);
        L.bq.pref = (uint16_t*)carve(b, 2ull * nw);
        L.bq.val = (float*)carve(b, 4ull * kMaxQ);
    }
    L.qv = (double*)carve(p, 8ull * 256);
    L.cut = nullptr;
    L.soff = nullptr;
    L.r = nullptr;
    L.ord = nullptr;
    L.wp0 = (uint32_t*)carve(p, 4ull * kMaxW);
    L.wlen = (uint32_t*)carve(p, 4ull * kMaxW);
    L.wst = (uint32_t*)carve(p, 4ull * (kMaxW + 1));
    L.scratch = (uint32_t*)carve(p, 4ull * (NT / kWave + 8));
    L.misc = (uint32_t*)carve(p, 4ull * 16);
    top.s0 = (float*)carve(p, 4ull * k);
    top.s1 = (float*)carve(p, 4ull * k);
    top.i0 = (uint32_t*)carve(p, 4ull * k);
    top.i1 = (uint32_t*)carve(p, 4ull * k);
    top.scratch = L.scratch;
    top.which = 0;
    top.hn = 0;
    top.k = k;
    uint8_t* u = p;
    uint8_t* q = u;
    L.q_term = (uint16_t*)carve(q, 2ull * kMaxQ);
    L.q_half = (uint16_t*)carve(q, 2ull * kMaxQ);
    L.A = nullptr;
    L.B = nullptr;
    q = u;
    L.cacc = (double*)carve(q, 8ull * NT);
    L.crs = (uint64_t*)carve(q, 8ull * NT);
    L.cdoc = (uint32_t*)carve(q, 4ull * NT);
    L.clen = (uint32_t*)carve(q, 4ull * NT);
    L.cslot = (uint8_t*)carve(q, 1ull * NT);
    top.cs = (float*)L.crs;                  // [NT] floats, then
    top.cid = (uint32_t*)(top.cs + NT);      // [NT] ids: 8 * NT bytes, as crs
}

size_t wide_eval_smem_bytes(uint32_t dim, uint32_t k) {
    constexpr size_t NT = kWideChunk;
    size_t s = region_bytes_for(dim) + r16u(8 * 256);
    s += 2 * r16u(4 * kMaxW) + r16u(4 * (kMaxW + 1)) + r16u(4 * (NT / kWave + 8)) + r16u(64);
    s += 4 * r16u(4 * (size_t)k);
    const size_t ingest = 2 * 2 * (size_t)kMaxQ + 32, gath = NT * (8 + 8 + 4 + 4 + 1) + 6 * 16;
    return s + (ingest > gath ? ingest : gath);
}

template <int NT>
size_t search_smem_bytes_t(uint32_t dim, uint32_t P, uint32_t k) {
    size_t s = region_bytes_for(dim);
    s += r16u(8 * 256) + r16u(2 * kMaxQ);
    s += r16u(4 * ((size_t)P + 1)) + r16u(4 * (size_t)P) + r16u(2 * (size_t)P);
    s += 2 * r16u(4 * kMaxW) + r16u(4 * (kMaxW + 1)) + r16u(4 * (NT / kWave + 8)) + r16u(64);
    s += 4 * r16u(4 * (size_t)k) + 2 * r16u(4 * (size_t)NT);
    s += union_bytes<NT>(P);
    return s;
}

// Query value of term t as fp64 (0 when absent): u8 slot table ...
struct LookU8 {
    const uint8_t* slot;
    const double* qv;
    __device__ __forceinline__ double operator()(uint32_t t) const { return qv[slot[t]]; }
};

// ... or membership bitmap with prefix counts (long queries).
struct LookBits {
    QTable q;
    __device__ __forceinline__ double operator()(uint32_t t) const {
        float v;
        return q_lookup(q, t, v) ? (double)v : 0.0;
    }
};

// One 16-byte group of 8 summary entries starting at entry eb: adds
// sum(q) and sum(q * code) of the entries inside [S0, S1) to the LDS
// accumulators of their blocks.
template <int NT, typename Look>
__device__ __forceinline__ void summary_group(const SearchLds<NT>& L, const Look& look, uint64_t eb, uint4 tv,
                                              uint2 cv, uint64_t S0, uint64_t S1, uint32_t nb) {
    const uint32_t tw[4] = {tv.x, tv.y, tv.z, tv.w};
    const uint32_t lo = (uint32_t)((eb > S0 ? eb : S0) - S0);
    uint32_t blo = 0, bhi = nb;  // block holding entry lo
    while (bhi - blo > 1) {
        const uint32_t mid = (blo + bhi) >> 1;
        if (L.soff[mid] <= lo) blo = mid; else bhi = mid;
    }
    uint32_t blk = blo;
    if (eb >= S0 && eb + 8 <= S1 && L.soff[blk + 1] >= lo + 8) {
        // the whole group lies inside one block: straight-line
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e) {
            const double qd = look((tw[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu);
            const uint32_t code = ((e < 4 ? cv.x : cv.y) >> ((e & 3) * 8)) & 0xFFu;
            sa += qd;
            sb = fma(qd, (double)code, sb);  // exact: 11 x 8 bits
        }
        if (sa != 0.0) { atomicAdd(&L.A[blk], sa); atomicAdd(&L.B[blk], sb); }
        return;
    }
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (uint32_t e = 0; e < 8; ++e) {
        if (eb + e < S0 || eb + e >= S1) continue;
        const uint32_t rel = (uint32_t)(eb + e - S0);
        while (L.soff[blk + 1] <= rel) {
            if (sa != 0.0) { atomicAdd(&L.A[blk], sa); atomicAdd(&L.B[blk], sb); }
            sa = 0.0; sb = 0.0;
            ++blk;
        }
        const double qd = look((tw[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu);
        const uint32_t code = ((e < 4 ? cv.x : cv.y) >> ((e & 3) * 8)) & 0xFFu;
        sa += qd;
        sb = fma(qd, (double)code, sb);
    }
    if (sa != 0.0) { atomicAdd(&L.A[blk], sa); atomicAdd(&L.B[blk], sb); }
}

// Gather documents [0, tot) of the current window (slot s covers
// [wst[s], wst[s+1]); big_off offsets the postings of a single oversized
// block) and score them.  A thread per document fetches its posting and row
// offsets; then groups of kLanesPerDoc lanes own whole rows, two documents
// per group at a time, reading each row as 16-byte aligned groups of 4 words
// (words outside the row are replaced by 0, which adds exactly 0) with
// kUnroll loads per document in flight, and reduce with shuffles.  On return
// cacc[t] is the exact score of document t (fp64) and clen[t] its number of
// nonzeros.  Every thread calls it; it ends with a barrier.  BR: the
// window's list has block-major copies of its rows (16-byte aligned,
// zero-padded: no masking needed), posting p's at copy p + cbias.
template <int NT, typename Look, bool BR>
__device__ inline void gather_and_score_t(const DevIdx& ix, const SearchLds<NT>& L, const Look& look, uint32_t tot,
                                          uint32_t nwb, uint32_t big_off, int64_t cbias) {
    const int tid = threadIdx.x;
    if ((uint32_t)tid < tot) {
        uint32_t s = 0;
        while (s + 1 < nwb && L.wst[s + 1] <= (uint32_t)tid) ++s;
        const uint32_t p = L.wp0[s] + big_off + ((uint32_t)tid - L.wst[s]);
        const uint32_t d = ix.postings[p];
        uint64_t rs;
        uint32_t len;
        if (BR) {  // block-major copy: contiguous with its neighbours, 16-byte aligned
            const uint64_t c = (uint64_t)((int64_t)p + cbias);
            rs = ix.prow[c] << 2;
            len = ix.pnnz[c];
        } else {
            rs = ix.row_ptr[d];
            len = (uint32_t)(ix.row_ptr[d + 1] - rs);
        }
        L.cdoc[tid] = d;
        L.crs[tid] = rs;
        L.clen[tid] = len;
        L.cslot[tid] = (uint8_t)s;
    }
    __syncthreads();
    const uint32_t* src = BR ? ix.brow : ix.words;
    constexpr uint32_t G = kLanesPerDoc, NG = NT / kLanesPerDoc, H = kDocsPerGroup;
    const uint32_t grp = (uint32_t)tid / G, gl = (uint32_t)tid % G;
    for (uint32_t base = grp; base < tot; base += H * NG) {
        uint64_t g0[H];
        uint32_t ng[H], head[H], len[H];
        double acc[H];
        uint32_t ngmax = 0;
#pragma unroll
        for (uint32_t h = 0; h < H; ++h) {
            const uint32_t t = base + h * NG;
            const uint64_t rs = t < tot ? L.crs[t] : 0;
            len[h] = t < tot ? L.clen[t] : 0;
            g0[h] = rs >> 2;
            head[h] = (uint32_t)(rs & 3);  // row start inside its first group
            ng[h] = len[h] ? (uint32_t)(((rs + len[h] + 3) >> 2) - g0[h]) : 0u;
            ngmax = max(ngmax, ng[h]);
            acc[h] = 0.0;
        }
        for (uint32_t k = gl; k < ngmax; k += kUnroll * G) {
            uint4 w[H][kUnroll];
#pragma unroll
            for (uint32_t h = 0; h < H; ++h)
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u)
                    w[h][u] = (k + u * G < ng[h]) ? *(const uint4*)(src + ((g0[h] + k + u * G) << 2))
                                                 : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (uint32_t h = 0; h < H; ++h)
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    // position of the group's first word relative to the row start
                    const int32_t rel = (int32_t)((k + u * G) * 4u) - (int32_t)head[h];
                    const uint32_t ww[4] = {w[h][u].x, w[h][u].y, w[h][u].z, w[h][u].w};
#pragma unroll
                    for (uint32_t e = 0; e < 4; ++e) {
                        const int32_t at = rel + (int32_t)e;
                        const uint32_t x = (BR || (at >= 0 && at < (int32_t)len[h])) ? ww[e] : 0u;
                        acc[h] = fma(look(x & 0xFFFFu), (double)half_bits_to_float(x >> 16), acc[h]);
                    }
                }
        }
#pragma unroll
        for (uint32_t h = 0; h < H; ++h) acc[h] = group_sum<double, G>(acc[h]);
        if (gl == 0) {
#pragma unroll
            for (uint32_t h = 0; h < H; ++h)
                if (base + h * NG < tot) L.cacc[base + h * NG] = acc[h];
        }
    }
    __syncthreads();
}

// Offset from a posting of a block to its block-major copy (bc = bcopy of
// the block, p0 = its first posting), or kNoBias when its list has none.
constexpr int64_t kNoBias = INT64_MIN;
__device__ __forceinline__ int64_t copy_bias(uint32_t bc, uint32_t p0) {
    return bc == kNoCopy ? kNoBias : (int64_t)bc - (int64_t)p0;
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint64_t u = (uint64_t)x;
    return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32)) << 32) |
                     (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)u));
}

// cbias: copy_bias of the window's list (the same for all its blocks).
template <int NT, typename Look>
__device__ inline void gather_and_score(const DevIdx& ix, const SearchLds<NT>& L, const Look& look, uint32_t tot,
                                        uint32_t nwb, uint32_t big_off, int64_t cbias) {
    if (cbias != kNoBias)
        gather_and_score_t<NT, Look, true>(ix, L, look, tot, nwb, big_off, cbias);
    else
        gather_and_score_t<NT, Look, false>(ix, L, look, tot, nwb, big_off, 0);
}

// Fold the gathered documents of window slot `slot` (all of them when
// slot < 0) into the top-k.  Every thread calls it.
template <int NT>
__device__ inline void fold_slot(const SearchLds<NT>& L, TopK<NT>& top, uint32_t tot, int slot, uint64_t& c_nnz) {
    const int tid = threadIdx.x;
    bool cand = false;
    float sc = 0.0f;
    uint32_t d = 0;
    if ((uint32_t)tid < tot && (slot < 0 || L.cslot[tid] == (uint32_t)slot)) {
        sc = (float)L.cacc[tid];
        d = L.cdoc[tid];
        c_nnz += L.clen[tid];
        cand = top.admits(sc, d);
    }
    uint32_t nc;
    const uint32_t at = block_exscan<NT>(cand ? 1u : 0u, L.scratch, &nc);
    if (cand) { top.cs[at] = sc; top.cid[at] = d; }
    __syncthreads();
    if (nc) top.merge(nc);
}

// fold_slot for the wide traversal's stored candidate sets (no nonzero
// counts): returns after one barrier when no candidate of the slot enters.
template <int NT>
__device__ inline void fold_slot_sparse(const SearchLds<NT>& L, TopK<NT>& top, uint32_t tot, int slot) {
    const int tid = threadIdx.x;
    bool cand = false;
    float sc = 0.0f;
    uint32_t d = 0;
    if ((uint32_t)tid < tot && (slot < 0 || L.cslot[tid] == (uint32_t)slot)) {
        sc = (float)L.cacc[tid];
        d = L.cdoc[tid];
        cand = top.admits(sc, d);
    }
    if (!__syncthreads_or(cand ? 1 : 0)) return;
    uint32_t nc;
    const uint32_t at = block_exscan<NT>(cand ? 1u : 0u, L.scratch, &nc);
    if (cand) { top.cs[at] = sc; top.cid[at] = d; }
    __syncthreads();
    top.merge(nc);
}

// fold_slot_sparse for window slots [0, m) at once.
template <int NT>
__device__ inline void fold_prefix_sparse(const SearchLds<NT>& L, TopK<NT>& top, uint32_t tot, uint32_t m) {
    const int tid = threadIdx.x;
    bool cand = false;
    float sc = 0.0f;
    uint32_t d = 0;
    if ((uint32_t)tid < tot && L.cslot[tid] < m) {
        sc = (float)L.cacc[tid];
        d = L.cdoc[tid];
        cand = top.admits(sc, d);
    }
    if (!__syncthreads_or(cand ? 1 : 0)) return;
    uint32_t nc;
    const uint32_t at = block_exscan<NT>(cand ? 1u : 0u, L.scratch, &nc);
    if (cand) { top.cs[at] = sc; top.cid[at] = d; }
    __syncthreads();
    top.merge(nc);
}

// Learned-probe decision for one block.  Kept out of line (the search's
// register budget is set by its gather phase); the parameter pointer is
// made wave-uniform and read through the constant address space, so the
// 449 parameters come in with scalar loads.
typedef const double __attribute__((address_space(4)))* ConstDoublePtr;

__device__ __noinline__ bool probe_keeps(const double* w, double tau, float r, double h0, uint32_t n_docs,
                                         uint32_t n_q, uint32_t ci) {
    const uint64_t pv = (uint64_t)w;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)pv);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(pv >> 32));
    const ConstDoublePtr W = (ConstDoublePtr)((hi << 32) | lo);
    double f[kProbeIn];
    probe_features(r, h0, n_docs, n_q, ci, f);
    double z = W[kProbeB2];
    for (uint32_t l = 0; l < kProbeHidden; ++l) {
        double x = W[kProbeB1 + l];
#pragma unroll
        for (uint32_t i = 0; i < kProbeIn; ++i) x = fma(W[l * kProbeIn + i], f[i], x);
        z = fma(W[kProbeW2 + l], probe_q(x, 0x1p-8, 256.0), z);
    }
    return z >= tau;
}

// The whole window (every gathered document) folded into the idle buffer of
// the top-k without making it live; returns merge_pending's count.
template <int NT>
__device__ inline uint32_t fold_window_pending(const SearchLds<NT>& L, TopK<NT>& top, uint32_t tot, uint64_t& c_nnz) {
    const int tid = threadIdx.x;
    bool cand = false;
    float sc = 0.0f;
    uint32_t d = 0;
    if ((uint32_t)tid < tot) {
        sc = (float)L.cacc[tid];
        d = L.cdoc[tid];
        c_nnz += L.clen[tid];
        cand = top.admits(sc, d);
    }
    uint32_t nc;
    const uint32_t at = block_exscan<NT>(cand ? 1u : 0u, L.scratch, &nc);
    if (cand) { top.cs[at] = sc; top.cid[at] = d; }
    __syncthreads();
    return nc ? top.merge_pending(nc) : 0u;
}

// Step 2a for the nb blocks of a list (first block b0, summary entries
// [S0, S1)): per block, sum(q) in L.A and sum(q * code) in L.B.  Every
// thread calls it; it ends with a barrier.
template <int NT, typename Look>
__device__ __forceinline__ void summary_sums(const DevIdx& ix, const SearchLds<NT>& L, const Look& look, uint32_t b0,
                                             uint32_t nb, uint64_t S0, uint64_t S1) {
    const int tid = threadIdx.x;
    for (uint32_t i = tid; i <= nb; i += NT) L.soff[i] = (uint32_t)(ix.blk_sum_off[b0 + i] - S0);
    for (uint32_t i = tid; i < nb; i += NT) { L.A[i] = 0.0; L.B[i] = 0.0; }
    __syncthreads();
    const uint64_t gend = (S1 + 7) >> 3;
    for (uint64_t g0 = (S0 >> 3) + tid; g0 < gend; g0 += (uint64_t)NT * kSumUnroll) {
        uint4 tv[kSumUnroll];
        uint2 cv[kSumUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kSumUnroll; ++u) {
            const uint64_t g = g0 + (uint64_t)u * NT;
            if (g < gend) {
                tv[u] = *(const uint4*)(ix.sum_term + (g << 3));
                cv[u] = *(const uint2*)(ix.sum_code + (g << 3));
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kSumUnroll; ++u) {
            const uint64_t g = g0 + (uint64_t)u * NT;
            if (g < gend) summary_group<NT, Look>(L, look, g << 3, tv[u], cv[u], S0, S1, nb);
        }
    }
    __syncthreads();
}

// Bitonic sort of (L.r, L.ord)[0, Pl) into (r desc, ord asc) order; Pl is a
// power of two.  Every thread calls it; it ends with a barrier when Pl > 1.
template <int NT>
__device__ __forceinline__ void sort_blocks(const SearchLds<NT>& L, uint32_t Pl) {
    const int tid = threadIdx.x;
    for (uint32_t kk = 2; kk <= Pl; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = tid; i < Pl; i += NT) {
                const uint32_t l = i ^ jj;
                if (l > i) {
                    const float ri = L.r[i], rl = L.r[l];
                    const uint32_t oi = L.ord[i], ol = L.ord[l];
                    const bool l_first = rl > ri || (rl == ri && ol < oi);
                    if (((i & kk) == 0) ? l_first : !l_first) {
                        L.r[i] = rl; L.r[l] = ri; L.ord[i] = (uint16_t)ol; L.ord[l] = (uint16_t)oi;
                    }
                }
            }
            __syncthreads();
        }
    }
}

struct Counters {
    uint64_t sum = 0, blocks = 0, eval = 0, docs = 0, tests = 0, nnz = 0;
};

// List-major schedule: the top-k and counters a query carries from one cut
// position to the next.
__device__ __forceinline__ uint32_t carry_in(const SearchArgs& a, float* s0, uint32_t* i0, uint32_t qi) {
    const uint32_t hn = a.ls_hn[qi];
    for (uint32_t i = threadIdx.x; i < hn; i += blockDim.x) {
        s0[i] = a.ls_hs[(size_t)qi * a.k + i];
        i0[i] = a.ls_hid[(size_t)qi * a.k + i];
    }
    return hn;
}

// Adds the counters of the earlier positions (thread 0's C and nnz); if
// the query has later positions, stores its top-k and counters for them.
__device__ __forceinline__ void carry_out(const SearchArgs& a, const float* H, const uint32_t* I, uint32_t hn,
                                       uint32_t qi, bool last, Counters& C, unsigned long long& nnz) {
    uint64_t* cc = a.ls_cnt + (size_t)qi * 6;
    if (a.pos > 0 && threadIdx.x == 0) {
        C.sum += cc[0]; C.blocks += cc[1]; C.eval += cc[2]; C.docs += cc[3]; nnz += cc[4]; C.tests += cc[5];
    }
    if (last) return;
    for (uint32_t i = threadIdx.x; i < hn; i += blockDim.x) {
        a.ls_hs[(size_t)qi * a.k + i] = H[i];
        a.ls_hid[(size_t)qi * a.k + i] = I[i];
    }
    if (threadIdx.x == 0) {
        a.ls_hn[qi] = hn;
        cc[0] = C.sum; cc[1] = C.blocks; cc[2] = C.eval; cc[3] = C.docs; cc[4] = nnz; cc[5] = C.tests;
    }
}

// Steps 2a-2c for the cut lists ci0 .. ci1 - 1 of query qi.  WIDE: the
// wide schedule's traversal (sorted summary scores and the speculated
// blocks' top-k sets come from the list and evaluation passes).
template <int NT, typename Look, bool WIDE>
__device__ __forceinline__ void run_lists(const SearchArgs& a, const SearchLds<NT>& L, TopK<NT>& top, const Look& look, uint32_t qi,
                          uint32_t ci0, uint32_t ci1, uint32_t nvalid, Counters& C) {
    const int tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t W = a.window;
    if constexpr (WIDE) {
        // the headers of all cut lists in one round of loads
        for (uint32_t ci = ci0 + tid; ci < ci1; ci += NT) {
            const uint32_t t = L.cut[ci];
            const uint32_t b0 = ix.list_off[t], b1 = ix.list_off[t + 1];
            L.wl_b0[ci] = b0;
            L.wl_nb[ci] = b1 - b0;
            L.wl_S0[ci] = ix.blk_sum_off[b0];
            L.wl_S1[ci] = ix.blk_sum_off[b1];
            L.wl_D[ci] = b1 > b0 ? a.wd_nspec[(size_t)qi * a.cmax + ci] : 0u;
            uint32_t bc = kNoCopy, bp = 0;
            if (ix.bcopy && b1 > b0) {  // both loads in one round
                bc = ix.bcopy[b0];
                bp = ix.blk_post_off[b0];
            }
            L.wl_cb[ci] = copy_bias(bc, bp);
        }
        __syncthreads();
    }
    for (uint32_t ci = ci0; ci < ci1; ++ci) {
        const uint32_t t = L.cut[ci];
        uint32_t b0, b1;
        if constexpr (WIDE) {
            b0 = L.wl_b0[ci];
            b1 = b0 + L.wl_nb[ci];
        } else {
            b0 = ix.list_off[t];
            b1 = ix.list_off[t + 1];
        }
        const uint32_t nb = b1 - b0;
        if (tid == 0 && ci < a.prefix_stride) {
            if (a.list_term) a.list_term[(size_t)qi * a.prefix_stride + ci] = t;
            if (a.list_hmin) a.list_hmin[(size_t)qi * a.prefix_stride + ci] = top.full() ? top.min_score() : -1.0f;
        }
        if (nb == 0) {
            if (a.prefix && tid == 0 && ci < a.prefix_stride) a.prefix[(size_t)qi * a.prefix_stride + ci] = 0;
            continue;
        }
        // ---------------------------------------- a. summary scores
        uint64_t S0, S1;
        int64_t cbias;  // block-major copies of the list's rows, if any
        if constexpr (WIDE) {
            S0 = L.wl_S0[ci];
            S1 = L.wl_S1[ci];
            cbias = uniform64(L.wl_cb[ci]);
        } else {
            S0 = ix.blk_sum_off[b0];
            S1 = ix.blk_sum_off[b1];
            const uint32_t ub0 = __builtin_amdgcn_readfirstlane(b0);
            const uint32_t bc = ix.bcopy ? ix.bcopy[ub0] : kNoCopy;
            cbias = copy_bias(bc, ix.blk_post_off[ub0]);
        }
        C.sum += S1 - S0;
        C.blocks += nb;
        [[maybe_unused]] const float* wr = nullptr;     // WIDE: sorted scores of this list
        [[maybe_unused]] const uint16_t* wo = nullptr;  // WIDE: their block indexes
        [[maybe_unused]] uint32_t D = 0;                // WIDE: speculated blocks (sorted positions [0, D))
        [[maybe_unused]] size_t wslot = 0;              // WIDE: result slot of sorted position 0
        if constexpr (WIDE) {
            const size_t lb = ((size_t)qi * a.cmax + ci) * a.sort_cap;
            wr = a.wd_r + lb;
            wo = a.wd_ord + lb;
            D = L.wl_D[ci];
            wslot = ((size_t)qi * a.cmax + ci) * a.depth;
        } else {
            summary_sums<NT, Look>(ix, L, look, b0, nb, S0, S1);
        }
        // ---------------------------------------- b. prefilter + sort
        // (WIDE: the scores arrive sorted, so the survivors of the
        // heap_factor rule are a prefix; L.ord holds sorted positions)
        const bool full0 = top.full();
        const double hmin0 = full0 ? (double)top.min_score() : 0.0;
        const bool learned = full0 && a.probe_w != nullptr;
        uint32_t nsurv = 0;
        // the list's posting offsets, loaded once for all its windows into
        // soff (the summary offsets are dead from here on): block j holds
        // postings [soff[j], soff[j + 1])
        if (tid == 0) L.soff[nb] = ix.blk_post_off[b0 + nb];
        for (uint32_t c = 0; c < nb; c += NT) {
            const uint32_t i = c + tid;
            float rv = 0.0f;
            bool keep = false;
            if (i < nb) {
                L.soff[i] = ix.blk_post_off[b0 + i];
                uint32_t bi = i;
                if constexpr (WIDE) {
                    rv = wr[i];
                    bi = wo[i];
                    if (i < D) {
                        L.wfirst[i] = a.wd_first[wslot + i];
                        L.wdocs[i] = a.wd_docs[wslot + i];
                        L.wnnz[i] = a.wd_nnz[wslot + i];
                    }
                } else {
                    rv = (float)((double)ix.blk_m[b0 + i] * L.A[i] + (double)ix.blk_delta[b0 + i] * L.B[i]);
                }
                if (learned) {
                    keep = probe_keeps(a.probe_w, a.tau, rv, hmin0, ix.blk_post_off[b0 + bi + 1] - ix.blk_post_off[b0 + bi],
                                       nvalid, ci);
                } else {
                    keep = !(full0 && (double)rv * (double)a.hf < hmin0);
                }
            }
            uint32_t cnt;
            const uint32_t at = block_exscan<NT>(keep ? 1u : 0u, L.scratch, &cnt);
            if (keep) { L.r[nsurv + at] = rv; L.ord[nsurv + at] = (uint16_t)i; }
            nsurv += cnt;
        }
        uint32_t Pl = 2;
        while (Pl < nsurv) Pl <<= 1;
        for (uint32_t i = nsurv + tid; i < Pl; i += NT) { L.r[i] = -INFINITY; L.ord[i] = 0xFFFFu; }
        __syncthreads();
        if (!WIDE && nsurv > 1 && !learned) sort_blocks<NT>(L, Pl);
        // ---------------------------------------- c. traversal
        uint32_t pos = 0, evaluated = 0;
        bool stop = false;
        while (pos < nsurv && !stop) {
            uint32_t nwb = 0, tot = 0;
            [[maybe_unused]] bool spec = false;   // WIDE: a window of speculated blocks
            [[maybe_unused]] uint32_t wdocs = 0;  // WIDE: documents of the window's blocks
            [[maybe_unused]] uint64_t wnnz = 0;   // WIDE: their nonzeros (speculated blocks)
            if constexpr (WIDE) spec = L.ord[pos] < D;
            if (spec) {
                // consecutive speculated blocks; their chunks' stored top-k
                // sets are the candidates, which yields the same top-k as all
                // of their documents (a document outside its chunk's k best
                // has k better ones in the same block)
                const uint32_t k = a.k;
                // wave 0 forms the window: consecutive speculated blocks while
                // their candidates fit (a speculated block alone always does),
                // the first candidate of each (wst), their sizes and items
                if (tid < kWave) {
                    const uint32_t s = (uint32_t)tid;
                    const bool in = s < kMaxW && pos + s < nsurv;
                    const uint32_t o = in ? L.ord[pos + s] : 0u;
                    const bool sp = in && o < D;
                    const uint32_t c = sp ? (L.wdocs[o] + kWideChunk - 1) / kWideChunk * k : 0u;
                    const uint64_t nsp = __ballot(!sp);
                    const uint32_t run = nsp ? (uint32_t)__ffsll((unsigned long long)nsp) - 1u : (uint32_t)kWave;
                    uint32_t incl = c;
#pragma unroll
                    for (int d = 1; d < kWave; d <<= 1) {
                        const uint32_t y = __shfl_up(incl, d, kWave);
                        if (s >= (uint32_t)d) incl += y;
                    }
                    const bool take = s < run && (s == 0 || incl <= (uint32_t)NT);
                    const uint32_t n = (uint32_t)__popcll(__ballot(take));
                    const uint32_t total = __shfl(incl, (int)(n > 0 ? n - 1 : 0), kWave);
                    const uint64_t nnz_s = take ? L.wnnz[o] : 0ull;
                    const uint32_t docs_s = take ? L.wdocs[o] : 0u;
                    if (take) {
                        L.wst[s] = incl - c;
                        L.wlen[s] = docs_s;
                        L.crs[s] = nnz_s;
                        L.wp0[s] = L.wfirst[o];
                    }
                    const unsigned long long wn = wave_sum((unsigned long long)nnz_s);
                    const uint32_t wd = (uint32_t)wave_sum((unsigned long long)docs_s);
                    if (s == 0) {
                        L.wst[n] = total;
                        L.misc[12] = n;
                        L.misc[13] = total;
                        L.misc[14] = wd;
                        L.crs[kMaxW] = wn;
                    }
                }
                __syncthreads();
                nwb = __builtin_amdgcn_readfirstlane(L.misc[12]);
                tot = __builtin_amdgcn_readfirstlane(L.misc[13]);
                wdocs = L.misc[14];
                wnnz = L.crs[kMaxW];
                if ((uint32_t)tid < tot) {
                    uint32_t lo = 0, hi = nwb;  // last block with wst <= tid
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (L.wst[mid] <= (uint32_t)tid) lo = mid; else hi = mid;
                    }
                    const size_t e = (size_t)L.wp0[lo] * k + ((uint32_t)tid - L.wst[lo]);
                    L.cacc[tid] = (double)a.wd_ps[e];
                    L.cdoc[tid] = a.wd_pid[e];
                    L.clen[tid] = 0;
                    L.cslot[tid] = (uint8_t)lo;
                }
                __syncthreads();
            } else {
            if ((uint32_t)tid < W && pos + tid < nsurv) {
                uint32_t j;
                if constexpr (WIDE) j = wo[L.ord[pos + tid]];
                else j = L.ord[pos + tid];
                const uint32_t p0 = L.soff[j];
                L.wp0[tid] = p0;
                L.wlen[tid] = L.soff[j + 1] - p0;
            }
            __syncthreads();
            for (uint32_t s = 0; s < W && pos + s < nsurv; ++s) {
                const uint32_t len = L.wlen[s];
                if (s > 0 && tot + len > (uint32_t)NT) break;
                tot += len;
                ++nwb;
            }
            if (tot > (uint32_t)NT) {
                // a single block larger than a chunk: evaluated alone
                if (!learned && top.full()) {
                    ++C.tests;
                    if ((double)L.r[pos] * (double)a.hf < (double)top.min_score()) { stop = true; break; }
                }
                ++evaluated;
                C.docs += tot;
                for (uint32_t c0 = 0; c0 < tot; c0 += NT) {
                    const uint32_t n = min((uint32_t)NT, tot - c0);
                    if (tid == 0) { L.wst[0] = 0; L.wst[1] = n; }
                    __syncthreads();
                    gather_and_score<NT, Look>(ix, L, look, n, 1, c0, cbias);
                    fold_slot<NT>(L, top, n, -1, C.nnz);
                }
                ++pos;
                __syncthreads();
                continue;
            }
            if (tid == 0) {
                uint32_t run = 0;
                for (uint32_t s = 0; s < nwb; ++s) { L.wst[s] = run; run += L.wlen[s]; }
                L.wst[nwb] = run;
            }
            __syncthreads();
            gather_and_score<NT, Look>(ix, L, look, tot, nwb, 0, cbias);
            wdocs = tot;
            }
            if constexpr (WIDE) {
                if (spec && !learned && !top.full()) {
                    // Blocks folded before the top-k fills are not tested: fold
                    // them at once.  While it is not full every positive id
                    // not yet held enters, and a block's chunk sets hold all
                    // its positive documents or at least k, so counting their
                    // new ids finds the first block tested, f, exactly.
                    uint32_t* cnt = L.wp0;  // free once the candidates are loaded
                    if ((uint32_t)tid < kMaxW) cnt[tid] = 0;
                    __syncthreads();
                    if ((uint32_t)tid < tot) {
                        const float sc = (float)L.cacc[tid];
                        const uint32_t d = L.cdoc[tid];
                        bool fresh = sc > 0.0f;
                        if (fresh && top.hn > 0) {
                            const uint32_t r = top.rank_in_heap(sc, d);
                            fresh = !(r < top.hn && top.hs()[r] == sc && top.hid()[r] == d);
                        }
                        if (fresh) atomicAdd(&cnt[L.cslot[tid]], 1u);
                    }
                    __syncthreads();
                    uint32_t run = top.hn, f = 0;
                    while (f < nwb && run < a.k) run += cnt[f++];
                    fold_prefix_sparse<NT>(L, top, tot, f);
                    evaluated += f;
                    for (uint32_t s = 0; s < f; ++s) {
                        C.docs += L.wlen[s];
                        if (tid == 0) C.nnz += L.crs[s];
                    }
                    pos += f;  // the rest of the window starts with a full top-k
                    __syncthreads();
                    continue;
                }
            }
            // Whole-window fold.  A probe-owned list makes no decisions.  With
            // the heap_factor rule and a heap already full, fold everything
            // into the idle buffer: heap.min only grows while the window is
            // replayed, so if even the window's last (smallest r) block passes
            // against the merged minimum, every block passes in order and the
            // merged set is the sequential result.  Otherwise replay block by
            // block from the unchanged live set.
            bool folded = false;
            if (learned) {
                evaluated += nwb;
                if constexpr (WIDE) {
                    C.docs += wdocs;
                    if (tid == 0) C.nnz += wnnz;
                } else {
                    C.docs += tot;
                }
                if (WIDE && spec)
                    fold_slot_sparse<NT>(L, top, tot, -1);
                else
                    fold_slot<NT>(L, top, tot, -1, C.nnz);
                folded = true;
            } else if (nwb > 1 && top.full() && (double)L.r[pos] * (double)a.hf >= (double)top.min_score() &&
                       (!WIDE || (double)L.r[pos + nwb - 1] * (double)a.hf >= (double)top.min_score())) {
                // (wide: skipped when the last block already fails against the
                // current minimum, since the merged one is not smaller)
                uint64_t nnz = 0;
                const uint32_t ns = fold_window_pending<NT>(L, top, tot, nnz);
                const float m2 = ns ? top.pending_min() : top.min_score();
                if ((double)L.r[pos + nwb - 1] * (double)a.hf >= (double)m2) {
                    top.commit(ns);
                    evaluated += nwb;
                    C.tests += nwb;
                    C.nnz += nnz;
                    if constexpr (WIDE) {
                        C.docs += wdocs;
                        if (tid == 0) C.nnz += wnnz;
                    } else {
                        C.docs += tot;
                    }
                    folded = true;
                }
            }
            for (uint32_t s = 0; s < nwb && !folded; ++s) {
                if (!learned && top.full()) {
                    ++C.tests;
                    if ((double)L.r[pos + s] * (double)a.hf < (double)top.min_score()) { stop = true; break; }
                }
                ++evaluated;
                C.docs += L.wlen[s];
                if constexpr (WIDE)
                    if (spec && tid == 0) C.nnz += L.crs[s];
                if (WIDE && spec)
                    fold_slot_sparse<NT>(L, top, tot, (int)s);
                else
                    fold_slot<NT>(L, top, tot, (int)s, C.nnz);
            }
            pos += stop ? 0u : nwb;
            __syncthreads();
        }
        if (learned) C.tests += nb;                     // one probe decision per block
        else if (!stop && nsurv < nb) ++C.tests;        // the first dropped block ends the list
        if (a.prefix && tid == 0 && ci < a.prefix_stride)
            a.prefix[(size_t)qi * a.prefix_stride + ci] = (uint16_t)min(evaluated, 65535u);
        C.eval += evaluated;
        __syncthreads();
    }
}

// Step 1 for query qi: validation flags, the term lookup in LDS (u8 slot
// table, or bitmap + prefix counts + values for long queries) and, with CUT,
// the cut lists in L.cut.  Every thread calls it; it ends with a barrier.
struct Ingested {
    uint64_t q0;      // first word of the query's row
    uint32_t nqe;     // words read (at most kMaxQ)
    uint32_t nvalid;  // valid distinct terms
    uint32_t ncut;    // cut lists (CUT only, else 0)
    uint32_t status;  // SEISMIC_QSTATUS_* bits
    bool u8mode;      // slot table (else bitmap)
};

template <int NT, bool CUT>
__device__ __forceinline__ Ingested ingest_query(const SearchArgs& a, const SearchLds<NT>& L, uint32_t qi, uint32_t nw) {
    const int tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    const uint64_t raw = q1 - q0;
    const uint32_t nqe = (uint32_t)min<uint64_t>(raw, (uint64_t)kMaxQ);
    if (tid < 12) L.misc[tid] = 0;  // 8..9: query mass (fp64), 10: alpha_q-MSS size
    __syncthreads();
    uint32_t st = (raw > (uint64_t)kMaxQ) ? 4u : 0u;
    for (uint32_t j = tid; j < nqe; j += NT) {
        const uint32_t w = a.q_words[q0 + j];
        const uint32_t t = w & 0xFFFFu, h = w >> 16;
        bool keep = true;
        if (t >= ix.dim) { st |= 1u; keep = false; }
        if (!half_ok(h)) { st |= 8u; keep = false; }
        if (j > 0 && t <= (a.q_words[q0 + j - 1] & 0xFFFFu)) st |= 2u;
        if (keep) {
            const uint64_t bit = 1ull << (t & 63u);
            const uint64_t old = atomicOr((unsigned long long*)&L.bq.bits[t >> 6], (unsigned long long)bit);
            if (old & bit) st |= 2u;  // repeated term
        }
        L.q_term[j] = keep ? (uint16_t)t : (uint16_t)0xFFFFu;
        L.q_half[j] = (uint16_t)h;
    }
    if (st) atomicOr(&L.misc[0], st);
    __syncthreads();
    if (L.misc[0] & 2u) {
        // terms not strictly ascending (unsorted or repeated): the row is
        // answered as an empty query, whatever order the entries came in;
        // the bits it set are cleared with the slot table below
        for (uint32_t j = tid; j < nqe; j += NT) L.q_term[j] = 0xFFFFu;
        __syncthreads();
    }
    build_prefix<NT>(L.bq.bits, L.bq.pref, nw, L.scratch);
    uint32_t nvalid_local = 0;
    double mass_local = 0.0;
    for (uint32_t j = tid; j < nqe; j += NT) {
        const bool v = L.q_term[j] != 0xFFFFu;
        nvalid_local += v ? 1u : 0u;
        if (v) mass_local += (double)half_bits_to_float(L.q_half[j]);
    }
    if (nvalid_local) atomicAdd(&L.misc[1], nvalid_local);
    // every fp16 value is a multiple of 2^-24 below 2^16, so partial sums of
    // at most kMaxQ of them are multiples of 2^-24 below 2^26: exact in
    // fp64 in any order (the same holds for the "before" sums of the cut)
    if (a.qmass > 0.0 && mass_local != 0.0) atomicAdd((double*)&L.misc[8], mass_local);
    __syncthreads();
    const uint32_t nvalid = __builtin_amdgcn_readfirstlane(L.misc[1]);
    const bool u8mode = nvalid <= kMaxSlots;
    const uint32_t ncut0 = (a.cut == 0 || a.cut > nvalid) ? nvalid : a.cut;
    const double mass_target = a.qmass * *(const double*)&L.misc[8];
    (void)mass_target;
    // slot of every valid entry (1-based rank of its term)
    uint32_t my_slot[kMaxQ / NT];
#pragma unroll
    for (uint32_t r = 0; r < kMaxQ / NT; ++r) {
        const uint32_t j = tid + r * NT;
        my_slot[r] = 0;
        if (j >= nqe) continue;
        const uint32_t t = L.q_term[j];
        if (t == 0xFFFFu) continue;
        const uint64_t w = L.bq.bits[t >> 6];
        const uint32_t slot = L.bq.pref[t >> 6] + (uint32_t)__popcll(w & ((1ull << (t & 63u)) - 1ull));
        my_slot[r] = slot + 1;
        if (u8mode) L.qv[slot + 1] = (double)half_bits_to_float(L.q_half[j]);
    }
    if constexpr (CUT) {
        // cut order: value desc (positive fp16: bit order), then term asc.
        // With alpha_q > 0 the cut also stops at the alpha_q-MSS of the query:
        // an entry belongs to it while the mass ranked before it is below
        // alpha_q * ||q||_1 (exact fp64 sums).
        uint32_t in_mss = 0;
        for (uint32_t j = tid; j < nqe; j += NT) {
            const uint32_t t = L.q_term[j];
            if (t == 0xFFFFu) continue;
            const uint32_t h = L.q_half[j];
            uint32_t rank = 0;
            double before = 0.0;
            for (uint32_t i = 0; i < nqe; ++i) {
                const uint32_t ti = L.q_term[i];
                const uint32_t hi = L.q_half[i];
                const bool b = ti != 0xFFFFu && (hi > h || (hi == h && ti < t));
                rank += b ? 1u : 0u;
                if (b && a.qmass > 0.0) before += (double)half_bits_to_float(hi);
            }
            if (rank < ncut0) L.cut[rank] = (uint16_t)t;
            if (a.qmass > 0.0 && before < mass_target) ++in_mss;
        }
        if (in_mss) atomicAdd(&L.misc[10], in_mss);
    }
    const uint32_t status = __builtin_amdgcn_readfirstlane(L.misc[0]);
    __syncthreads();
    const uint32_t ncut = CUT ? __builtin_amdgcn_readfirstlane(a.qmass > 0.0 ? min(ncut0, L.misc[10]) : ncut0) : 0u;
    if (u8mode) {
        // bitmap + prefix -> slot table
        for (uint32_t i = tid; i < (10 * nw + 15) / 16; i += NT) ((uint4*)L.region)[i] = make_uint4(0, 0, 0, 0);
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kMaxQ / NT; ++r)
            if (my_slot[r]) L.region[L.q_term[tid + r * NT]] = (uint8_t)my_slot[r];
    } else {
#pragma unroll
        for (uint32_t r = 0; r < kMaxQ / NT; ++r)
            if (my_slot[r]) L.bq.val[my_slot[r] - 1] = half_bits_to_float(L.q_half[tid + r * NT]);
    }
    __syncthreads();
    return Ingested{q0, nqe, nvalid, ncut, status, u8mode};
}

// Step 1 for a row the list pass found valid, strictly ascending and of at
// most kMaxSlots terms: entry j's term has slot j + 1, so the slot table and
// the slot values are written straight from the row, with none of
// ingest_query's checks and scans.  Every thread calls it; it ends with a
// barrier; restore_region undoes it.
template <int NT>
__device__ __forceinline__ Ingested ingest_direct(const SearchArgs& a, const SearchLds<NT>& L, uint32_t qi) {
    const int tid = threadIdx.x;
    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    const uint32_t n = (uint32_t)min<uint64_t>(q1 - q0, (uint64_t)kMaxSlots);
    for (uint32_t j = tid; j < n; j += NT) {
        const uint32_t w = a.q_words[q0 + j];
        L.region[w & 0xFFFFu] = (uint8_t)(j + 1);
        L.qv[j + 1] = (double)half_bits_to_float(w >> 16);
    }
    __syncthreads();
    return Ingested{q0, n, n, 0u, 0u, true};
}

// Puts the lookup region of an ingested query back to all-zero.
template <int NT>
__device__ __forceinline__ void restore_region(const SearchArgs& a, const SearchLds<NT>& L, const Ingested& in) {
    const int tid = threadIdx.x;
    if (in.u8mode) {
        for (uint32_t j = tid; j < in.nqe; j += NT) {
            const uint32_t t = a.q_words[in.q0 + j] & 0xFFFFu;
            if (t < a.ix.dim) L.region[t] = 0;
        }
    } else {
        for (uint32_t i = tid; i < L.region_bytes / 16; i += NT) ((uint4*)L.region)[i] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
}

// LIST: the list-major schedule's per-position kernel (a separate instance, so that
// the query-major kernel carries none of its code; its carry code would
// take it past three workgroups per CU, so the bound keeps three and the
// compiler spills a few values of that code).
template <int NT, bool LIST, bool WIDE = false>
__global__ __launch_bounds__(NT, (LIST && NT == 256) ? 3 : 1) void k_search(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t nw = (ix.dim + 63u) / 64u;
    SearchLds<NT> L;
    TopK<NT> top;
    [[maybe_unused]] uint8_t* end = carve_lds<NT>(smem, ix.dim, a.sort_cap, a.k, L, top);
    if constexpr (WIDE) {
        L.wfirst = (uint32_t*)carve(end, 4ull * kWideMaxDepth);
        L.wdocs = (uint32_t*)carve(end, 4ull * kWideMaxDepth);
        L.wnnz = (uint64_t*)carve(end, 8ull * kWideMaxDepth);
        L.wl_b0 = (uint32_t*)carve(end, 4ull * kWideMaxCut);
        L.wl_nb = (uint32_t*)carve(end, 4ull * kWideMaxCut);
        L.wl_D = (uint32_t*)carve(end, 4ull * kWideMaxCut);
        L.wl_S0 = (uint64_t*)carve(end, 8ull * kWideMaxCut);
        L.wl_S1 = (uint64_t*)carve(end, 8ull * kWideMaxCut);
        L.wl_cb = (int64_t*)carve(end, 8ull * kWideMaxCut);
    }
    for (uint32_t i = tid; i < L.region_bytes / 16; i += NT) ((uint4*)L.region)[i] = make_uint4(0, 0, 0, 0);
    if (tid == 0) L.qv[0] = 0.0;
    __syncthreads();

    const uint32_t nq = a.nq_dev ? min(*a.nq_dev, a.nq) : a.nq;
    // work items: queries, or at a list-major position the queries holding a
    // cut list at this position
    uint32_t it0 = 0, n_items = nq;
    if constexpr (LIST) {
        it0 = a.ls_seg[a.pos];
        n_items = a.ls_seg[a.pos + 1] - it0;
    }
    for (;;) {
        // ------------------------------------------------ next query
        if (tid == 0) L.misc[15] = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(L.misc[15]);
        if (item >= n_items) break;
        const uint32_t qi = __builtin_amdgcn_readfirstlane(LIST ? a.ls_items[it0 + item] : item);
        top.which = 0;
        top.hn = 0;

        Ingested in;
        uint32_t fast = 0;
        if constexpr (WIDE) fast = a.wd_fast[qi];
        if (fast) {  // the list pass checked the row and cut it
            in = ingest_direct<NT>(a, L, qi);
            in.ncut = fast - 1u;
            if ((uint32_t)tid < in.ncut) L.cut[tid] = (uint16_t)a.wd_cut[(size_t)qi * a.cmax + tid];
            __syncthreads();
        } else {
            in = ingest_query<NT, true>(a, L, qi, nw);
        }
        const uint32_t ncut = in.ncut, nvalid = in.nvalid, status = in.status;
        const bool u8mode = in.u8mode;

        uint32_t ci0 = 0, ci1 = ncut;
        bool last = true;
        if constexpr (LIST) {
            ci0 = min(a.pos, ncut);
            ci1 = min(a.pos + 1, ncut);
            last = a.pos + 1 >= ncut;
            if (a.pos > 0) {  // the top-k carried from the previous position
                top.hn = carry_in(a, top.s0, top.i0, qi);
                __syncthreads();
            }
        }

        Counters C;
        if (u8mode) {
            LookU8 look{L.region, L.qv};
            run_lists<NT, LookU8, WIDE>(a, L, top, look, qi, ci0, ci1, nvalid, C);
        } else {
            LookBits look{L.bq};
            run_lists<NT, LookBits, WIDE>(a, L, top, look, qi, ci0, ci1, nvalid, C);
        }
        unsigned long long nnz_tot = 0;
        if (a.counters || LIST) {
            const unsigned long long v = wave_sum((unsigned long long)C.nnz);
            unsigned long long* red = (unsigned long long*)L.crs;  // union region is free here
            if ((tid & (kWave - 1)) == 0) red[tid / kWave] = v;
            __syncthreads();
            for (int w = 0; w < NT / kWave; ++w) nnz_tot += red[w];
            __syncthreads();
        }
        if constexpr (LIST) {
            carry_out(a, top.hs(), top.hid(), top.hn, qi, last, C, nnz_tot);
            if (a.pos == 0) {  // the cut lists, for the items of the later positions
                if ((uint32_t)tid < ncut) a.ls_cut[(size_t)qi * a.cmax + tid] = L.cut[tid];
                if (tid == 0) a.ls_ncut[qi] = ncut;
            }
        }

        // ------------------------------------------------------------ output
        if (last) {
            const float* H = top.hs();
            const uint32_t* I = top.hid();
            for (uint32_t i = tid; i < a.k; i += NT) {
                const bool have = i < top.hn;
                a.out_ids[(size_t)qi * a.k + i] = have ? I[i] : 0xFFFFFFFFu;
                a.out_scores[(size_t)qi * a.k + i] = have ? H[i] : -INFINITY;
            }
            for (uint32_t i = ncut + tid; i < a.prefix_stride; i += NT) {
                if (a.prefix) a.prefix[(size_t)qi * a.prefix_stride + i] = 0;
                if (a.list_term) a.list_term[(size_t)qi * a.prefix_stride + i] = 0xFFFFFFFFu;
                if (a.list_hmin) a.list_hmin[(size_t)qi * a.prefix_stride + i] = -1.0f;
            }
            if (a.counters && tid == 0) {
                uint64_t* c = a.counters + (size_t)qi * 8;
                c[0] = C.sum; c[1] = C.blocks; c[2] = C.eval; c[3] = C.docs; c[4] = nnz_tot; c[5] = C.tests;
                c[6] = status; c[7] = ncut;
            }
        }
        restore_region<NT>(a, L, in);
    }
}

// Wide schedule, list pass: one (query, cut list) pair per item.  Scores
// the summaries of all blocks of the list (step 2a), sorts them by (r desc,
// block asc) (step 2b without the heap-dependent drop), stores the order,
// and enqueues the first `depth` blocks for the evaluation pass.
template <int NT>
__global__ __launch_bounds__(NT) void k_wide_lists(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t nw = (ix.dim + 63u) / 64u;
    SearchLds<NT> L;
    TopK<NT> top;
    carve_lds<NT>(smem, ix.dim, a.sort_cap, a.k, L, top);
    for (uint32_t i = tid; i < L.region_bytes / 16; i += NT) ((uint4*)L.region)[i] = make_uint4(0, 0, 0, 0);
    if (tid == 0) L.qv[0] = 0.0;
    __syncthreads();
    const uint32_t nq = a.nq_dev ? min(*a.nq_dev, a.nq) : a.nq;
    const uint32_t n_items = nq * a.cmax;
    for (;;) {
        if (tid == 0) L.misc[15] = atomicAdd(a.wd_cnt + 0, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(L.misc[15]);
        if (item >= n_items) break;
        const uint32_t qi = item / a.cmax, ci = item - qi * a.cmax;
        const Ingested in = ingest_query<NT, true>(a, L, qi, nw);
        if (ci >= in.ncut && tid == 0) a.wd_nspec[(size_t)qi * a.cmax + ci] = 0;  // past the cut: nothing speculated
        if (ci < in.ncut) {
            const uint32_t t = L.cut[ci];
            if (tid == 0) a.wd_cut[(size_t)qi * a.cmax + ci] = t;
            const uint32_t b0 = ix.list_off[t], nb = ix.list_off[t + 1] - b0;
            if (nb) {
                const uint64_t S0 = ix.blk_sum_off[b0], S1 = ix.blk_sum_off[b0 + nb];
                if (in.u8mode)
                    summary_sums<NT, LookU8>(ix, L, LookU8{L.region, L.qv}, b0, nb, S0, S1);
                else
                    summary_sums<NT, LookBits>(ix, L, LookBits{L.bq}, b0, nb, S0, S1);
                uint32_t Pl = 2;
                while (Pl < nb) Pl <<= 1;
                for (uint32_t i = tid; i < Pl; i += NT) {
                    if (i < nb) {
                        L.r[i] = (float)((double)ix.blk_m[b0 + i] * L.A[i] + (double)ix.blk_delta[b0 + i] * L.B[i]);
                        L.ord[i] = (uint16_t)i;
                    } else {
                        L.r[i] = -INFINITY;
                        L.ord[i] = 0xFFFFu;
                    }
                }
                __syncthreads();
                sort_blocks<NT>(L, Pl);
                const size_t lb = ((size_t)qi * a.cmax + ci) * a.sort_cap;
                for (uint32_t i = tid; i < nb; i += NT) {
                    a.wd_r[lb + i] = L.r[i];
                    a.wd_ord[lb + i] = L.ord[i];
                }
                // speculated blocks: the first D0 of the order, each split into
                // chunks of kWideChunk documents (one evaluation item each);
                // the list keeps the longest prefix whose items fit the item
                // capacity and whose blocks' chunk sets fit one traversal
                // window (chunks * k <= wd_nt candidates)
                const uint32_t D0 = min(nb, nq <= kWideTinyBatch ? a.depth : a.depth_large);
                uint32_t b = 0, n = 0, ch = 0, bc = kNoCopy;
                if ((uint32_t)tid < D0) {
                    b = b0 + L.ord[tid];
                    n = ix.blk_post_off[b + 1] - ix.blk_post_off[b];
                    if (ix.bcopy) bc = ix.bcopy[b];  // carried by the block's items
                    ch = (n + kWideChunk - 1) / kWideChunk;
                }
                uint32_t T;
                const uint32_t at = block_exscan<NT>(ch, L.scratch, &T);
                if (tid == 0) L.misc[14] = atomicAdd(a.wd_cnt + 1, T);
                __syncthreads();
                const uint32_t base = L.misc[14];
                const bool fits = (uint64_t)base + at + ch <= a.wd_icap && ch * a.k <= a.wd_nt;
                if (tid == 0) L.misc[13] = D0;
                __syncthreads();
                if ((uint32_t)tid < D0 && !fits) atomicMin(&L.misc[13], (uint32_t)tid);
                __syncthreads();
                const uint32_t D = L.misc[13];
                const uint32_t slot0 = (qi * a.cmax + ci) * a.depth;
                if (tid == 0) a.wd_nspec[(size_t)qi * a.cmax + ci] = D;
                if ((uint32_t)tid < D) {
                    a.wd_first[slot0 + tid] = base + at;
                    a.wd_nnz[slot0 + tid] = 0;
                    a.wd_docs[slot0 + tid] = n;
                    for (uint32_t j = 0; j < ch; ++j) a.wd_items[base + at + j] = make_uint4(b, j, slot0 + tid, bc);
                } else if ((uint32_t)tid < D0) {
                    // items reserved for blocks past the prefix: no-ops
                    for (uint32_t j = 0; j < ch; ++j)
                        if ((uint64_t)base + at + j < a.wd_icap) a.wd_items[base + at + j] = make_uint4(0xFFFFFFFFu, 0, 0, 0);
                }
            } else if (tid == 0) {
                a.wd_nspec[(size_t)qi * a.cmax + ci] = 0;
            }
        }
        if (ci == 0 && tid == 0) {
            a.wd_lb[qi] = 0.0f;  // the evaluation pass may raise it
            // a valid row of at most kMaxSlots terms: its slot table can be
            // written straight from the row (ingest_direct)
            a.wd_fast[qi] = (in.status == 0 && in.u8mode && in.nvalid == in.nqe) ? 1u + in.ncut : 0u;
        }
        restore_region<NT>(a, L, in);
    }
}

// Wide schedule, evaluation pass: one chunk of kWideChunk documents of a
// speculated block per item.  Scores the chunk's documents exactly (step
// 2c's gather) and stores their top-k beside the item; the block's
// nonzeros are summed with an atomic add.  A workgroup keeps the lookup of
// its last query.
__global__ __launch_bounds__(kWideChunk) void k_wide_eval(SearchArgs a) {
    constexpr int NT = kWideChunk;
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t nw = (ix.dim + 63u) / 64u;
    SearchLds<NT> L;
    TopK<NT> top;
    carve_lds_eval(smem, ix.dim, a.k, L, top);
    for (uint32_t i = tid; i < L.region_bytes / 16; i += NT) ((uint4*)L.region)[i] = make_uint4(0, 0, 0, 0);
    if (tid == 0) L.qv[0] = 0.0;
    __syncthreads();
    const uint32_t n_items = min(a.wd_cnt[1], a.wd_icap);
    const uint32_t nq = a.nq_dev ? min(*a.nq_dev, a.nq) : a.nq;
    const uint32_t per_query = a.cmax * a.depth;
    const uint32_t k = a.k;
    const bool bound = a.probe_w == nullptr;
    uint32_t cur = 0xFFFFFFFFu;
    Ingested in{};
    // The queue first hands out, for every query, the first chunk of the
    // first block of its first cut list (queue positions [0, nq)), then every
    // item in order (an item already handed out first is skipped).  That
    // block is evaluated with an empty heap, so every later prune decision
    // of the query sees a heap minimum at least the k-th best score of that
    // chunk: the query's bound, published once the chunk is scored.  An item
    // of a later block whose summary score r has r * hf below the bound is
    // pruned by the traversal before its candidates could be read, so it is
    // not scored.  A bound read before it is published is 0 (no skip).
    for (;;) {
        if (tid == 0) L.misc[15] = atomicAdd(a.wd_cnt + 2, 1u);
        __syncthreads();
        const uint32_t ticket = __builtin_amdgcn_readfirstlane(L.misc[15]);
        if (ticket >= nq + n_items) break;
        uint32_t item;
        const bool first = ticket < nq;
        if (first) {
            const size_t qc = (size_t)ticket * a.cmax;
            if (!bound || a.wd_nspec[qc] == 0) {
                __syncthreads();
                continue;
            }
            item = a.wd_first[qc * a.depth];
        } else {
            item = ticket - nq;
        }
        const uint4 it = a.wd_items[item];
        const uint32_t b = __builtin_amdgcn_readfirstlane(it.x);
        if (b == 0xFFFFFFFFu) {  // a reserved item left unused
            __syncthreads();
            continue;
        }
        const uint32_t c = __builtin_amdgcn_readfirstlane(it.y), slot = __builtin_amdgcn_readfirstlane(it.z);
        const uint32_t qi = slot / per_query;
        if (!first && bound) {
            const uint32_t lp = slot - qi * per_query, ci = lp / a.depth, pos = lp - ci * a.depth;
            if (ci == 0 && pos == 0 && c == 0) {  // handed out first
                __syncthreads();
                continue;
            }
            // the bound may be published while the waves of this workgroup
            // read it: one read, shared through LDS, keeps the decision (and
            // the barriers after it) the same for every wave
            if (tid == 0)
                L.misc[14] = __float_as_uint(__hip_atomic_load(a.wd_lb + qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            __syncthreads();
            const float lb = __uint_as_float(L.misc[14]);
            const float r = a.wd_r[((size_t)qi * a.cmax + ci) * a.sort_cap + pos];
            if ((ci > 0 || pos > 0) && (double)r * (double)a.hf < (double)lb) {
                for (uint32_t i = tid; i < k; i += NT) {
                    a.wd_ps[(size_t)item * k + i] = -INFINITY;
                    a.wd_pid[(size_t)item * k + i] = 0xFFFFFFFFu;
                }
                __syncthreads();
                continue;
            }
        }
        if (qi != cur) {
            if (cur != 0xFFFFFFFFu) restore_region<NT>(a, L, in);
            if (a.wd_fast[qi])
                in = ingest_direct<NT>(a, L, qi);
            else
                in = ingest_query<NT, false>(a, L, qi, nw);
            cur = qi;
        }
        top.which = 0;
        top.hn = 0;
        const uint32_t p0 = ix.blk_post_off[b], n = ix.blk_post_off[b + 1] - p0;
        const uint32_t c0 = c * NT, m = min((uint32_t)NT, n - c0);
        const int64_t cbias = copy_bias(__builtin_amdgcn_readfirstlane(it.w), p0);
        if (tid == 0) { L.wst[0] = 0; L.wst[1] = m; L.wp0[0] = p0; }
        __syncthreads();
        if (in.u8mode)
            gather_and_score<NT, LookU8>(ix, L, LookU8{L.region, L.qv}, m, 1, c0, cbias);
        else
            gather_and_score<NT, LookBits>(ix, L, LookBits{L.bq}, m, 1, c0, cbias);
        uint64_t nnz = 0;
        fold_slot<NT>(L, top, m, -1, nnz);
        const unsigned long long v = wave_sum((unsigned long long)nnz);
        unsigned long long* red = (unsigned long long*)L.crs;  // the gather arrays are free here
        if ((tid & (kWave - 1)) == 0) red[tid / kWave] = v;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < NT / kWave; ++w) tot += red[w];
            atomicAdd((unsigned long long*)(a.wd_nnz + slot), tot);
        }
        for (uint32_t i = tid; i < k; i += NT) {
            const bool have = i < top.hn;
            a.wd_ps[(size_t)item * k + i] = have ? top.hs()[i] : -INFINITY;
            a.wd_pid[(size_t)item * k + i] = have ? top.hid()[i] : 0xFFFFFFFFu;
        }
        if (first && tid == 0 && top.full())
            __hip_atomic_store(a.wd_lb + qi, top.min_score(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

__global__ void k_wide_reset(uint32_t* cnt, uint32_t* queue) {
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) *queue = 0;
}

__global__ void k_reset_queue(uint32_t* queue) {
    if (threadIdx.x == 0) *queue = 0;
}

// ----------------------------------------------- list-major schedule items
// Items are sorted by a key per (query, cut position): the rank of the
// position's list among all lists by block count (longest first), or dim
// for a query with no cut list (one item at position 0, which writes its
// empty result).  Counting sort over rows hist[r * (dim + 1) + key].
// Position 0's keys come from each query's largest entry (its first cut
// list); the later positions' from the cut lists that position 0 records.

__global__ __launch_bounds__(256) void k_items_zero(uint32_t* hist, uint32_t n) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_items_first(const uint32_t* nq_dev, uint32_t nq, const uint64_t* q_ptr,
                                                     const uint32_t* q_words, uint64_t q_nnz, uint32_t dim,
                                                     const uint32_t* term_rank, uint32_t* key0, uint32_t* hist) {
    const uint32_t n = nq_dev ? min(*nq_dev, nq) : nq;
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const uint64_t q1 = min(q_ptr[q + 1], q_nnz), q0 = min(q_ptr[q], q1);
    uint32_t bt = 0xFFFFFFFFu, bh = 0;
    for (uint64_t j = q0; j < min(q1, q0 + kMaxQ); ++j) {
        const uint32_t w = q_words[j], t = w & 0xFFFFu, h = w >> 16;
        if (t >= dim || !half_ok(h)) continue;
        if (bt == 0xFFFFFFFFu || h > bh || (h == bh && t < bt)) { bt = t; bh = h; }
    }
    const uint32_t key = bt == 0xFFFFFFFFu ? dim : term_rank[bt];
    key0[q] = key;
    atomicAdd(&hist[key], 1u);
}

__global__ __launch_bounds__(256) void k_items_count(const uint32_t* nq_dev, uint32_t nq, uint32_t cmax, uint32_t dim,
                                                     const uint16_t* cut, const uint32_t* ncut,
                                                     const uint32_t* term_rank, uint32_t* hist) {
    const uint32_t n = nq_dev ? min(*nq_dev, nq) : nq;
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const uint32_t c = min(ncut[q], cmax);
    for (uint32_t r = 1; r < c; ++r) atomicAdd(&hist[r * (dim + 1) + term_rank[cut[(size_t)q * cmax + r]]], 1u);
}

// Exclusive scan of rows [row0, row1) of hist in place (one workgroup),
// starting at seg[row0] (0 for row 0); seg[r] = first item of position r for
// r in [row0, row1]; the positions' queues zeroed.
__global__ __launch_bounds__(1024) void k_items_scan(uint32_t* hist, uint32_t row0, uint32_t row1, uint32_t dim,
                                                     uint32_t* seg, uint32_t* queues) {
    __shared__ uint32_t part[1024];
    const uint32_t tid = threadIdx.x, w = dim + 1, b = row0 * w, n = (row1 - row0) * w;
    const uint32_t base = row0 == 0 ? 0u : seg[row0];
    const uint32_t per = (n + 1023) / 1024, lo = min(n, tid * per), hi = min(n, lo + per);
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i) sum += hist[b + i];
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = base;
        for (uint32_t i = 0; i < 1024; ++i) { const uint32_t v = part[i]; part[i] = run; run += v; }
        seg[row1] = run;
    }
    __syncthreads();
    uint32_t run = part[tid];
    for (uint32_t i = lo; i < hi; ++i) {
        if (i % w == 0) seg[row0 + i / w] = run;
        const uint32_t v = hist[b + i];
        hist[b + i] = run;
        run += v;
    }
    for (uint32_t r = row0 + tid; r < row1; r += 1024) queues[r] = 0;
}

__global__ __launch_bounds__(256) void k_items_scatter(const uint32_t* nq_dev, uint32_t nq, uint32_t cmax,
                                                       uint32_t dim, const uint16_t* cut, const uint32_t* ncut,
                                                       const uint32_t* term_rank, const uint32_t* key0,
                                                       uint32_t* hist, uint32_t* items) {
    const uint32_t n = nq_dev ? min(*nq_dev, nq) : nq;
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    if (key0) {  // position 0
        items[atomicAdd(&hist[key0[q]], 1u)] = q;
        return;
    }
    const uint32_t c = min(ncut[q], cmax);
    for (uint32_t r = 1; r < c; ++r)
        items[atomicAdd(&hist[r * (dim + 1) + term_rank[cut[(size_t)q * cmax + r]]], 1u)] = q;
}

size_t search_smem_bytes(uint32_t nt, uint32_t dim, uint32_t sort_cap, uint32_t k) {
    if (nt == 1024) return search_smem_bytes_t<1024>(dim, sort_cap, k);
    return nt == 512 ? search_smem_bytes_t<512>(dim, sort_cap, k) : search_smem_bytes_t<256>(dim, sort_cap, k);
}

int wide_eval_blocks_per_cu(size_t smem) {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_wide_eval, kWideChunk, smem) == hipSuccess ? n : 0;
}

int search_blocks_per_cu(uint32_t nt, size_t smem) {
    int n = 0;
    hipError_t e = nt == 512 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<512, false>, 512, smem)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<256, false>, 256, smem);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_search(const SearchArgs& a, uint32_t nt, uint32_t grid, size_t smem, hipStream_t stream) {
    if (a.nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, stream, a.queue);
    if (nt == 512)
        hipLaunchKernelGGL((k_search<512, false>), dim3(grid), dim3(512), smem, stream, a);
    else
        hipLaunchKernelGGL((k_search<256, false>), dim3(grid), dim3(256), smem, stream, a);
    return hipGetLastError();
}

hipError_t launch_search_positions(SearchArgs a, const ListSched& ls, uint32_t nt, uint32_t grid, size_t smem,
                                hipStream_t stream) {
    if (a.nq == 0) return hipSuccess;
    const uint32_t cmax = a.cut, dim = a.ix.dim, qb = (a.nq + 255) / 256;
    a.mode = kModeList;
    a.cmax = cmax;
    a.ls_cut = ls.cut;
    a.ls_ncut = ls.ncut;
    a.ls_items = ls.items;
    a.ls_seg = ls.seg;
    a.ls_hs = ls.hs;
    a.ls_hid = ls.hid;
    a.ls_hn = ls.hn;
    a.ls_cnt = ls.cnt;
    const uint32_t hn = cmax * (dim + 1);
    auto position = [&](uint32_t r) {
        a.pos = r;
        a.queue = ls.queues + r;
        if (nt == 512)
            hipLaunchKernelGGL((k_search<512, true>), dim3(grid), dim3(512), smem, stream, a);
        else
            hipLaunchKernelGGL((k_search<256, true>), dim3(grid), dim3(256), smem, stream, a);
        return hipGetLastError();
    };
    hipLaunchKernelGGL(k_items_zero, dim3(std::min<uint32_t>(1024, (hn + 255) / 256)), dim3(256), 0, stream, ls.hist, hn);
    hipLaunchKernelGGL(k_items_first, dim3(qb), dim3(256), 0, stream, a.nq_dev, a.nq, a.q_ptr, a.q_words, a.q_nnz, dim,
                       ls.term_rank, ls.key0, ls.hist);
    hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, stream, ls.hist, 0u, 1u, dim, ls.seg, ls.queues);
    hipLaunchKernelGGL(k_items_scatter, dim3(qb), dim3(256), 0, stream, a.nq_dev, a.nq, cmax, dim, ls.cut, ls.ncut,
                       ls.term_rank, ls.key0, ls.hist, ls.items);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = position(0);
    if (e != hipSuccess || cmax < 2) return e;
    hipLaunchKernelGGL(k_items_count, dim3(qb), dim3(256), 0, stream, a.nq_dev, a.nq, cmax, dim, ls.cut, ls.ncut,
                       ls.term_rank, ls.hist);
    hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, stream, ls.hist, 1u, cmax, dim, ls.seg, ls.queues);
    hipLaunchKernelGGL(k_items_scatter, dim3(qb), dim3(256), 0, stream, a.nq_dev, a.nq, cmax, dim, ls.cut, ls.ncut,
                       ls.term_rank, (const uint32_t*)nullptr, ls.hist, ls.items);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (uint32_t r = 1; r < cmax && e == hipSuccess; ++r) e = position(r);
    return e;
}

hipError_t launch_search_wide(SearchArgs a, const WideSched& w, uint32_t nt, uint32_t grid, size_t smem,
                              uint32_t grid_lists, size_t smem_lists, uint32_t grid_eval, size_t smem_eval,
                              hipStream_t stream) {
    if (a.nq == 0) return hipSuccess;
    a.mode = kModeWide;
    a.cmax = a.cut;
    a.wd_r = w.r;
    a.wd_ord = w.ord;
    a.wd_nspec = w.nspec;
    a.wd_items = w.items;
    a.wd_icap = w.icap;
    a.wd_cnt = w.cnt;
    a.wd_first = w.first;
    a.wd_docs = w.docs;
    a.wd_nnz = w.nnz;
    a.wd_ps = w.ps;
    a.wd_pid = w.pid;
    a.wd_lb = w.lb;
    a.wd_fast = w.fast;
    a.wd_cut = w.cut;
    // the traversal's own window for blocks past the speculated ones
    a.window = nt == 512 ? 16u : 8u;
    a.wd_nt = nt;
    const uint32_t g_lists = std::min<uint64_t>(grid_lists, (uint64_t)a.nq * a.cmax);
    const uint32_t g_eval = std::min<uint64_t>(grid_eval, w.icap);
    const uint32_t g_fold = std::min<uint32_t>(grid, a.nq);
    hipLaunchKernelGGL(k_wide_reset, dim3(1), dim3(64), 0, stream, w.cnt, a.queue);
    if (nt == 512) {
        hipLaunchKernelGGL(k_wide_lists<kWideListThreads>, dim3(g_lists), dim3(kWideListThreads), smem_lists, stream, a);
        hipLaunchKernelGGL(k_wide_eval, dim3(g_eval), dim3(kWideChunk), smem_eval, stream, a);
        hipLaunchKernelGGL((k_search<512, false, true>), dim3(g_fold), dim3(512), smem + kWideMetaBytes, stream, a);
    } else {
        hipLaunchKernelGGL(k_wide_lists<kWideListThreads>, dim3(g_lists), dim3(kWideListThreads), smem_lists, stream, a);
        hipLaunchKernelGGL(k_wide_eval, dim3(g_eval), dim3(kWideChunk), smem_eval, stream, a);
        hipLaunchKernelGGL((k_search<256, false, true>), dim3(g_fold), dim3(256), smem + kWideMetaBytes, stream, a);
    }
    return hipGetLastError();
}

}  // namespace seismic_dev
