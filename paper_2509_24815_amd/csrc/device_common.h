// Device-side building blocks shared by the search and exact-search kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace seismic_dev {

constexpr int kWave = 64;
constexpr uint32_t kNoCopy = 0xFFFFFFFFu;

// The index as the kernels see it (all device pointers).
struct DevIdx {
    const uint64_t* row_ptr;
    const uint32_t* words;
    const uint32_t* list_off;
    const uint32_t* blk_post_off;
    const uint64_t* blk_sum_off;
    const float* blk_m;
    const float* blk_delta;
    const uint32_t* postings;
    const uint16_t* sum_term;  // padded to a multiple of 8 entries (+8)
    const uint8_t* sum_code;   // padded likewise
    // block-major copies of the rows of some or all lists (optional): block
    // b's postings have copies c = bcopy[b] + (p - blk_post_off[b]), or none
    // when bcopy[b] == kNoCopy (always the same for the blocks of one list);
    // copy c's row occupies 16-byte groups [prow[c], prow[c] + ceil(pnnz[c]
    // / 4)) of brow, zero-padded, and pnnz[c] is its number of nonzeros
    const uint32_t* bcopy;
    const uint64_t* prow;
    const uint32_t* pnnz;
    const uint32_t* brow;
    uint32_t dim;
    uint32_t n_docs;
};

__device__ __forceinline__ float half_bits_to_float(uint32_t h) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

__device__ __forceinline__ bool half_ok(uint32_t h) {
    return (h & 0x8000u) == 0 && ((h >> 10) & 0x1Fu) != 31u && (h & 0x7FFFu) != 0;
}

// Result order: larger score first, then smaller id.
__device__ __forceinline__ bool better(float s1, uint32_t d1, float s2, uint32_t d2) {
    return s1 > s2 || (s1 == s2 && d1 < d2);
}

__device__ __forceinline__ uint8_t* carve(uint8_t*& p, size_t bytes) {
    uint8_t* out = p;
    p += (bytes + 15) & ~size_t(15);
    return out;
}

// Query held in LDS as a membership bitmap over terms plus per-word prefix
// popcounts; the value of term t sits at slot pref[t/64] + popcount of the
// lower bits of bits[t/64].  Absent terms cost one LDS read.
struct QTable {
    uint64_t* bits;  // [nw]
    uint16_t* pref;  // [nw]
    float* val;      // [slots]
};

__device__ __forceinline__ bool q_lookup(const QTable& q, uint32_t t, float& v) {
    const uint64_t w = q.bits[t >> 6];
    const uint32_t b = t & 63u;
    if (!((w >> b) & 1ull)) return false;
    v = q.val[q.pref[t >> 6] + __popcll(w & ((1ull << b) - 1ull))];
    return true;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

template <typename T, int G>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Block-wide exclusive scan of one value per thread.  scratch needs
// NT/64 + 1 words.  Returns the exclusive prefix; *total gets the sum.
// Contains two barriers; every thread must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* scratch, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) scratch[wave] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        uint32_t c = scratch[w];
        base += (w < wave) ? c : 0u;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// Exclusive prefix popcounts of bits[0..nw) into pref (nw <= 16 * NT).
template <int NT>
__device__ inline void build_prefix(const uint64_t* bits, uint16_t* pref, uint32_t nw, uint32_t* scratch) {
    const uint32_t per = (nw + NT - 1) / NT;
    const uint32_t base = (uint32_t)threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (base + i < nw) local += (uint32_t)__popcll(bits[base + i]);
    uint32_t tot;
    uint32_t ex = block_exscan<NT>(local, scratch, &tot);
    for (uint32_t i = 0; i < per; ++i)
        if (base + i < nw) { pref[base + i] = (uint16_t)ex; ex += (uint32_t)__popcll(bits[base + i]); }
    __syncthreads();
}

// Sorted top-k set in LDS, double-buffered: (s0, i0) and (s1, i1); `which`
// selects the live copy.  hn entries are live, in result order.  merge()
// folds up to NT candidates into it, keeping the k best distinct ids.
// Every thread of the block calls merge with the same arguments.
template <int NT>
struct TopK {
    float* s0;
    float* s1;
    uint32_t* i0;
    uint32_t* i1;
    float* cs;       // [NT]: candidates, then the survivors compacted in place
    uint32_t* cid;   // [NT]
    uint32_t* scratch;  // [NT / 64 + 1]
    uint32_t which;
    uint32_t hn;
    uint32_t k;

    __device__ __forceinline__ const float* hs() const { return which ? s1 : s0; }
    __device__ __forceinline__ const uint32_t* hid() const { return which ? i1 : i0; }
    __device__ __forceinline__ bool full() const { return hn == k; }
    __device__ __forceinline__ float min_score() const { return hs()[k - 1]; }
    __device__ __forceinline__ uint32_t min_id() const { return hid()[k - 1]; }

    // number of live entries better than (s, d)
    __device__ __forceinline__ uint32_t rank_in_heap(float s, uint32_t d) const {
        const float* H = hs();
        const uint32_t* I = hid();
        uint32_t lo = 0, hi = hn;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (better(H[mid], I[mid], s, d)) lo = mid + 1; else hi = mid;
        }
        return lo;
    }

    // Would (s, d) enter the set right now (ignoring duplicates)?
    __device__ __forceinline__ bool admits(float s, uint32_t d) const {
        return s > 0.0f && (hn < k || better(s, d, min_score(), min_id()));
    }

    // Candidates in cs/cid[0..nc), written before a barrier.  Scores <= 0
    // are not results and are ignored; ids already present are skipped.
    __device__ void merge(uint32_t nc) { commit(merge_pending(nc)); }

    // Makes the set written by merge_pending live (ns = its return value).
    __device__ __forceinline__ void commit(uint32_t ns) {
        if (ns) {
            hn = min(k, hn + ns);
            which ^= 1u;
        }
    }

    // Smallest score of the pending set (ns > 0 and hn + ns >= k).
    __device__ __forceinline__ float pending_min() const { return (which ? s0 : s1)[k - 1]; }

    // merge() without making the result live: the merged set goes to the
    // idle buffer; returns the number of new entries (0: nothing written,
    // the live set is unchanged).
    __device__ uint32_t merge_pending(uint32_t nc) {
        const int tid = threadIdx.x;
        bool ok = false;
        float s = 0.0f;
        uint32_t d = 0;
        if ((uint32_t)tid < nc) {
            s = cs[tid];
            d = cid[tid];
            const uint32_t pos = rank_in_heap(s, d);
            const bool dup = pos < hn && hs()[pos] == s && hid()[pos] == d;
            ok = !dup && admits(s, d);
        }
        // every candidate is in registers before the scan's barriers, so
        // the survivors overwrite the candidate array
        uint32_t ns;
        const uint32_t at = block_exscan<NT>(ok ? 1u : 0u, scratch, &ns);
        float* ss = cs;
        uint32_t* sd = cid;
        if (ok) { ss[at] = s; sd[at] = d; }
        __syncthreads();
        if (ns == 0) return 0;
        const float* H = hs();
        const uint32_t* I = hid();
        float* NH = which ? s0 : s1;
        uint32_t* NI = which ? i0 : i1;
        for (uint32_t e = (uint32_t)tid; e < hn + ns; e += NT) {
            float es;
            uint32_t ed, rank;
            if (e < hn) {
                es = H[e]; ed = I[e];
                rank = e;
            } else {
                es = ss[e - hn]; ed = sd[e - hn];
                rank = rank_in_heap(es, ed);
            }
            for (uint32_t j = 0; j < ns; ++j)
                if (better(ss[j], sd[j], es, ed)) ++rank;
            if (rank < k) { NH[rank] = es; NI[rank] = ed; }
        }
        __syncthreads();
        return ns;
    }
};

}  // namespace seismic_dev
