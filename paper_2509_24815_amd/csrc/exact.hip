// Exact top-k (Definition "Sparse MIPS", Section 1.1) over a full inverted
// index.  One workgroup answers one query.  Documents are swept in ranges of
// kRange ids; for each range the postings of every query term that fall
// into it are accumulated into an LDS fp64 array (atomic adds: products are
// exact in fp32 and sums of values in [2^-6, 2^6] are exact in fp64, so the
// order does not matter), then the range's documents are offered to the
// LDS top-k in rounds of at most one candidate per thread.
//
// Per-term cursors only move forward.  The postings of a term inside a range
// are found with a window whose size adapts to the term's density; a window
// that ends before the range does is widened and the pass repeated for that
// term only.
#include "device_common.h"
#include "search_kernels.h"

namespace seismic_dev {

constexpr int kBlock = 256;
constexpr uint32_t kRange = 2048;
constexpr uint32_t kPost = 8;  // postings in flight per thread
constexpr uint32_t kInf = 0xFFFFFFFFu;

__device__ __forceinline__ uint8_t* xbump(uint8_t*& p, size_t bytes) {
    uint8_t* out = p;
    p += (bytes + 15) & ~size_t(15);
    return out;
}

// Exclusive scan of in[0..n) (n <= 1024) into out[0..n], out[n] = total.
__device__ inline uint32_t block_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* scratch) {
    const int tid = threadIdx.x;
    uint32_t base = (uint32_t)tid * 4u, loc[4], sum = 0;
    for (int i = 0; i < 4; ++i) { loc[i] = (base + i < n) ? in[base + i] : 0u; sum += loc[i]; }
    scratch[tid] = sum;
    __syncthreads();
    if (tid < kWave) {
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
        if (tid == kWave - 1) scratch[kBlock] = incl;
    }
    __syncthreads();
    uint32_t ex = scratch[tid];
    for (int i = 0; i < 4; ++i)
        if (base + i < n) { out[base + i] = ex; ex += loc[i]; }
    const uint32_t total = scratch[kBlock];
    if (tid == 0) out[n] = total;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kBlock) void k_exact(ExactArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const uint32_t qi = blockIdx.x;
    uint8_t* p = smem;
    double* acc = (double*)xbump(p, 8ull * kRange);
    uint64_t* cur = (uint64_t*)xbump(p, 8ull * kMaxQ);
    uint64_t* endp = (uint64_t*)xbump(p, 8ull * kMaxQ);
    uint32_t* win = (uint32_t*)xbump(p, 4ull * kMaxQ);
    uint32_t* wlen = (uint32_t*)xbump(p, 4ull * kMaxQ);
    uint32_t* pfx = (uint32_t*)xbump(p, 4ull * (kMaxQ + 1));
    uint32_t* fge = (uint32_t*)xbump(p, 4ull * kMaxQ);
    float* qv = (float*)xbump(p, 4ull * kMaxQ);
    uint32_t* scratch = (uint32_t*)xbump(p, 4ull * (kBlock + 1));
    uint32_t* misc = (uint32_t*)xbump(p, 4ull * 8);
    TopK<kBlock> top;
    top.s0 = (float*)xbump(p, 4ull * a.k);
    top.s1 = (float*)xbump(p, 4ull * a.k);
    top.i0 = (uint32_t*)xbump(p, 4ull * a.k);
    top.i1 = (uint32_t*)xbump(p, 4ull * a.k);
    top.cs = (float*)xbump(p, 4ull * kBlock);
    top.cid = (uint32_t*)xbump(p, 4ull * kBlock);
    top.scratch = scratch;
    top.which = 0;
    top.hn = 0;
    top.k = a.k;

    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    uint32_t nt = (uint32_t)min<uint64_t>(q1 - q0, (uint64_t)kMaxQ);
    // a row whose terms are not strictly ascending is answered as an empty
    // query, as the search does
    if (tid == 0) misc[1] = 0;
    __syncthreads();
    bool unsorted = false;
    for (uint32_t j = 1 + tid; j < nt; j += kBlock)
        unsorted |= (a.q_words[q0 + j] & 0xFFFFu) <= (a.q_words[q0 + j - 1] & 0xFFFFu);
    if (unsorted) misc[1] = 1;
    __syncthreads();
    if (misc[1]) nt = 0;
    for (uint32_t j = tid; j < nt; j += kBlock) {
        const uint32_t w = a.q_words[q0 + j];
        const uint32_t t = w & 0xFFFFu, h = w >> 16;
        if (t < a.dim && half_ok(h)) {
            cur[j] = a.csc_off[t];
            endp[j] = a.csc_off[t + 1];
            qv[j] = half_bits_to_float(h);
        } else {
            cur[j] = endp[j] = 0;
            qv[j] = 0.0f;
        }
        win[j] = 8;
    }
    __syncthreads();

    for (uint32_t s = 0; s < a.n_docs; s += kRange) {
        const uint32_t e = min(s + kRange, a.n_docs);
        for (uint32_t i = tid; i < kRange; i += kBlock) acc[i] = 0.0;
        for (uint32_t j = tid; j < nt; j += kBlock)
            wlen[j] = cur[j] < endp[j] ? (uint32_t)min<uint64_t>(win[j], endp[j] - cur[j]) : 0u;
        __syncthreads();
        for (;;) {
            for (uint32_t j = tid; j < nt; j += kBlock) fge[j] = kInf;
            if (tid == 0) misc[0] = 0;
            const uint32_t T = block_scan(wlen, pfx, nt, scratch);  // ends with a barrier
            if (T == 0) break;
            // term of the first item of this thread, then walk forward
            uint32_t j = 0;
            if ((uint32_t)tid < T) {
                uint32_t lo = 0, hi = nt;  // last j with pfx[j] <= tid
                while (hi - lo > 1) { uint32_t mid = (lo + hi) >> 1; if (pfx[mid] <= (uint32_t)tid) lo = mid; else hi = mid; }
                j = lo;
            }
            // kPost postings per thread per step: all their loads are issued
            // before any is consumed
            for (uint32_t i0 = tid; i0 < T; i0 += kBlock * kPost) {
                uint32_t dd[kPost], jj[kPost], oo[kPost];
                uint16_t vv[kPost];
#pragma unroll
                for (uint32_t u = 0; u < kPost; ++u) {
                    const uint32_t i = i0 + u * kBlock;
                    dd[u] = kInf;
                    if (i < T) {
                        while (pfx[j + 1] <= i) ++j;
                        jj[u] = j;
                        oo[u] = i - pfx[j];
                        const uint64_t pos = cur[j] + oo[u];
                        dd[u] = a.csc_doc[pos];
                        vv[u] = a.csc_val[pos];
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kPost; ++u) {
                    if (i0 + u * kBlock >= T) break;
                    if (dd[u] < e) {
                        atomicAdd(&acc[dd[u] - s], (double)(qv[jj[u]] * half_bits_to_float(vv[u])));
                    } else {
                        atomicMin(&fge[jj[u]], oo[u]);
                    }
                }
            }
            __syncthreads();
            for (uint32_t jj = tid; jj < nt; jj += kBlock) {
                const uint32_t w = wlen[jj];
                if (w == 0) continue;
                const uint32_t f = fge[jj];
                if (f != kInf) {
                    cur[jj] += f;
                    win[jj] = max(8u, f + f / 2u + 8u);
                    wlen[jj] = 0;
                } else {
                    cur[jj] += w;
                    if (cur[jj] < endp[jj]) {  // window ended before the range did
                        win[jj] = min(2u * win[jj], 1u << 20);
                        wlen[jj] = (uint32_t)min<uint64_t>(win[jj], endp[jj] - cur[jj]);
                        misc[0] = 1;
                    } else {
                        wlen[jj] = 0;
                    }
                }
            }
            __syncthreads();
            if (misc[0] == 0) break;
            __syncthreads();
        }
        // offer the range's documents, at most one per thread per round
        for (;;) {
            const float hmin_s = top.full() ? top.min_score() : 0.0f;
            const uint32_t hmin_d = top.full() ? top.min_id() : 0u;
            float bs = 0.0f;
            uint32_t bi = kInf;
            for (uint32_t i = tid; i < e - s; i += kBlock) {
                const float sc = (float)acc[i];
                if (!(sc > 0.0f)) continue;
                if (top.hn == top.k && !better(sc, s + i, hmin_s, hmin_d)) continue;
                if (bi == kInf || better(sc, s + i, bs, s + bi)) { bs = sc; bi = i; }
            }
            const bool has = bi != kInf;
            if (has) acc[bi] = 0.0;
            top.cs[tid] = bs;
            top.cid[tid] = has ? s + bi : 0u;
            const uint64_t m = __ballot(has);
            if ((tid & (kWave - 1)) == 0) scratch[tid / kWave] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t tot = 0;
            for (int w = 0; w < kBlock / kWave; ++w) tot += scratch[w];
            if (tot == 0) break;
            __syncthreads();  // everyone has read scratch before merge reuses it
            top.merge(kBlock);
        }
        __syncthreads();
    }
    for (uint32_t i = tid; i < a.k; i += kBlock) {
        const bool have = i < top.hn;
        a.out_ids[(size_t)qi * a.k + i] = have ? top.hid()[i] : 0xFFFFFFFFu;
        a.out_scores[(size_t)qi * a.k + i] = have ? top.hs()[i] : -INFINITY;
    }
}

size_t exact_smem_bytes(uint32_t k) {
    auto r16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    size_t s = r16(8ull * kRange) + 2 * r16(8ull * kMaxQ) + 2 * r16(4ull * kMaxQ) + r16(4ull * (kMaxQ + 1));
    s += 2 * r16(4ull * kMaxQ) + r16(4ull * (kBlock + 1)) + r16(32);
    s += 4 * r16(4ull * k) + 2 * r16(4ull * kBlock);
    return s;
}

hipError_t launch_exact(const ExactArgs& a, uint32_t nq, size_t smem, hipStream_t stream) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_exact, dim3(nq), dim3(kBlock), smem, stream, a);
    return hipGetLastError();
}

}  // namespace seismic_dev
