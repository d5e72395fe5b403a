// Device-side building blocks shared by the search and exact-search kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace seismic_dev {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kWave = 64;

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
    const uint16_t* sum_term;
    const uint8_t* sum_code;
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

// Exclusive prefix popcounts of bits[0..nw) into pref, by the whole block.
// nw <= 1024.  Ends with a barrier.
__device__ inline void build_prefix(const uint64_t* bits, uint16_t* pref, uint32_t nw, uint32_t* scratch) {
    const int tid = threadIdx.x;
    // each thread owns up to 4 consecutive words
    uint32_t base = (uint32_t)tid * 4u, local = 0;
    for (uint32_t i = 0; i < 4; ++i)
        if (base + i < nw) local += (uint32_t)__popcll(bits[base + i]);
    scratch[tid] = local;
    __syncthreads();
    if (tid < kWave) {  // wave 0 scans the 256 partial sums, 4 per lane
        uint32_t s[4], run = 0;
        for (int i = 0; i < 4; ++i) { s[i] = scratch[tid * 4 + i]; run += s[i]; }
        uint32_t incl = run;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            uint32_t y = __shfl_up(incl, o, kWave);
            if (tid >= o) incl += y;
        }
        uint32_t ex = incl - run;
        for (int i = 0; i < 4; ++i) { uint32_t v = s[i]; scratch[tid * 4 + i] = ex; ex += v; }
    }
    __syncthreads();
    uint32_t ex = scratch[tid];
    for (uint32_t i = 0; i < 4; ++i)
        if (base + i < nw) { pref[base + i] = (uint16_t)ex; ex += (uint32_t)__popcll(bits[base + i]); }
    __syncthreads();
}

// Sorted top-k set in LDS: hs/hid hold hn entries in result order.  merge()
// folds up to kBlock candidates (distinct ids, not yet filtered) into it and
// keeps the k best distinct ids.  Called by the whole block; all threads must
// pass the same (nc, k, hn).  Double-buffered: the caller swaps via `cur`.
struct TopK {
    float* hs[2];
    uint32_t* hid[2];
    float* cs;       // [kBlock] candidate scores
    uint32_t* cid;   // [kBlock] candidate ids
    uint32_t* flag;  // [kBlock + 32]
    int cur;
    uint32_t hn;
    uint32_t k;

    __device__ __forceinline__ uint32_t lower_pos(float s, uint32_t d) const {
        // number of heap entries better than (s, d)
        const float* H = hs[cur];
        const uint32_t* I = hid[cur];
        uint32_t lo = 0, hi = hn;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (better(H[mid], I[mid], s, d)) lo = mid + 1; else hi = mid;
        }
        return lo;
    }

    // Candidates are in cs/cid[0..nc); the caller put them there and issued a
    // barrier.  Candidates with a score <= 0 are ignored (not results).
    __device__ void merge(uint32_t nc) {
        const int tid = threadIdx.x;
        bool ok = false;
        float s = 0.0f;
        uint32_t d = 0;
        if ((uint32_t)tid < nc) {
            s = cs[tid];
            d = cid[tid];
            uint32_t pos = lower_pos(s, d);
            bool dup = pos < hn && hs[cur][pos] == s && hid[cur][pos] == d;
            ok = s > 0.0f && !dup && (hn < k || better(s, d, hs[cur][hn - 1], hid[cur][hn - 1]));
        }
        // compact survivors with a block-wide exclusive scan of ok
        const int lane = tid & (kWave - 1), wave = tid / kWave;
        uint64_t m = __ballot(ok);
        uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) flag[kBlock + wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t wbase = 0, ns = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            uint32_t c = flag[kBlock + w];
            if (w < wave) wbase += c;
            ns += c;
        }
        // survivors go to the top of the candidate arrays' second half
        float* ss = cs + kBlock;
        uint32_t* sd = cid + kBlock;
        if (ok) { ss[wbase + before] = s; sd[wbase + before] = d; }
        __syncthreads();
        if (ns == 0) return;
        const float* H = hs[cur];
        const uint32_t* I = hid[cur];
        float* NH = hs[cur ^ 1];
        uint32_t* NI = hid[cur ^ 1];
        for (uint32_t e = (uint32_t)tid; e < hn + ns; e += kBlock) {
            float es;
            uint32_t ed, rank;
            if (e < hn) {
                es = H[e]; ed = I[e];
                rank = e;
            } else {
                es = ss[e - hn]; ed = sd[e - hn];
                rank = lower_pos(es, ed);
            }
            for (uint32_t j = 0; j < ns; ++j)
                if (better(ss[j], sd[j], es, ed)) ++rank;
            if (rank < k) { NH[rank] = es; NI[rank] = ed; }
        }
        __syncthreads();
        hn = min(k, hn + ns);
        cur ^= 1;
    }
};

}  // namespace seismic_dev
