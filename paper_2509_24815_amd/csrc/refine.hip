// Refinement with the kappa-NN graph (Section 4.3; the last block of
// Algorithm 2), run right after the search on its results.  One workgroup
// per query:
//   1. S = the query's result ids (the heap after the traversal);
//   2. candidates = the distinct neighbours of S's members that are not in S
//      (at most k * kappa <= kRefineThreads, a thread each);
//   3. a thread per candidate scores it exactly against the forward row
//      (fp64 sum of exact fp16 products; query values looked up by binary
//      search in the query's sorted terms, staged in LDS);
//   4. the new top-k = the k best of S and the positive-scored candidates by
//      (score desc, id asc): every entry counts the entries better than it
//      (all ids are distinct), which is its output position.
// No decision depends on the order of the candidates, so the result equals
// the sequential insertion of the algorithm.
#include "search_kernels.h"

namespace seismic_dev {

namespace {

__device__ __forceinline__ double q_value(const uint16_t* qt, const double* qv, uint32_t n, uint32_t t) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (qt[mid] < t) lo = mid + 1; else hi = mid;
    }
    return (lo < n && qt[lo] == t) ? qv[lo] : 0.0;
}

}  // namespace

__global__ __launch_bounds__(kRefineThreads) void k_refine(RefineArgs a) {
    constexpr uint32_t NT = kRefineThreads;
    __shared__ uint16_t qt[kMaxQ];
    __shared__ double qv[kMaxQ];
    __shared__ uint32_t S[NT];
    __shared__ float Ss[NT];
    __shared__ uint32_t cand[NT];
    __shared__ uint32_t eid[2 * NT];
    __shared__ float esc[2 * NT];
    __shared__ uint32_t scratch[NT / kWave + 1];
    __shared__ uint32_t hn_s;
    const uint32_t nq = a.nq_dev ? min(*a.nq_dev, a.nq) : a.nq;
    const uint32_t qi = blockIdx.x;
    if (qi >= nq) return;
    const uint32_t tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t k = a.k, kap = a.kappa;

    // results of the traversal (sorted, padding at the end)
    if (tid == 0) hn_s = 0;
    __syncthreads();
    if (tid < k) {
        const uint32_t id = a.ids[(size_t)qi * k + tid];
        S[tid] = id;
        Ss[tid] = a.scores[(size_t)qi * k + tid];
        if (id != 0xFFFFFFFFu) atomicMax(&hn_s, tid + 1);
    }
    // the query row, as in the search: entries with a term < dim and a
    // finite positive value
    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    const uint32_t n = (uint32_t)min<uint64_t>(q1 - q0, (uint64_t)kMaxQ);
    for (uint32_t j = tid; j < n; j += NT) {
        const uint32_t w = a.q_words[q0 + j];
        const uint32_t t = w & 0xFFFFu, h = w >> 16;
        qt[j] = (uint16_t)t;
        qv[j] = (t < ix.dim && half_ok(h)) ? (double)half_bits_to_float(h) : 0.0;
    }
    __syncthreads();
    const uint32_t hn = hn_s, m = hn * kap;

    // candidates: distinct neighbours outside S
    uint32_t v = 0xFFFFFFFFu;
    bool keep = false;
    if (tid < m) {
        v = a.knn[(size_t)S[tid / kap] * kap + tid % kap];
        keep = v < ix.n_docs;
        for (uint32_t h = 0; h < hn && keep; ++h) keep = S[h] != v;
    }
    cand[tid] = keep ? v : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t j = 0; j < tid && keep; ++j) keep = cand[j] != v;  // first occurrence wins
    uint32_t tot;
    const uint32_t at = block_exscan<NT>(keep ? 1u : 0u, scratch, &tot);
    if (keep) eid[hn + at] = v;
    if (tid < hn) { eid[tid] = S[tid]; esc[tid] = Ss[tid]; }
    __syncthreads();

    // exact scores of the candidates
    uint64_t nnz = 0;
    if (tid < tot) {
        const uint32_t d = eid[hn + tid];
        const uint64_t r0 = ix.row_ptr[d], r1 = ix.row_ptr[d + 1];
        double acc = 0.0;
        for (uint64_t j = r0; j < r1; ++j) {
            const uint32_t x = ix.words[j];
            acc = fma(q_value(qt, qv, n, x & 0xFFFFu), (double)half_bits_to_float(x >> 16), acc);
        }
        esc[hn + tid] = (float)acc;
        nnz = r1 - r0;
    }
    __syncthreads();

    // top-k of S and the candidates: rank of each entry = entries better than it
    const uint32_t ne = hn + tot;
    uint32_t rank[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};
    float rs[2] = {0.0f, 0.0f};
    uint32_t rid[2] = {0u, 0u};
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t e = tid + r * NT;
        if (e >= ne || !(esc[e] > 0.0f)) continue;
        rs[r] = esc[e];
        rid[r] = eid[e];
        uint32_t c = 0;
        for (uint32_t o = 0; o < ne; ++o)
            c += (esc[o] > 0.0f && (esc[o] > rs[r] || (esc[o] == rs[r] && eid[o] < rid[r]))) ? 1u : 0u;
        rank[r] = c;
    }
    uint32_t npos;
    (void)block_exscan<NT>((rank[0] != 0xFFFFFFFFu ? 1u : 0u) + (rank[1] != 0xFFFFFFFFu ? 1u : 0u), scratch, &npos);
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r)
        if (rank[r] < k) {
            a.ids[(size_t)qi * k + rank[r]] = rid[r];
            a.scores[(size_t)qi * k + rank[r]] = rs[r];
        }
    for (uint32_t i = npos + tid; i < k; i += NT) {
        a.ids[(size_t)qi * k + i] = 0xFFFFFFFFu;
        a.scores[(size_t)qi * k + i] = -INFINITY;
    }
    if (a.counters) {
        const unsigned long long sn = wave_sum((unsigned long long)nnz);
        __shared__ unsigned long long red[NT / kWave];
        if ((tid & (kWave - 1)) == 0) red[tid / kWave] = sn;
        __syncthreads();
        if (tid == 0) {
            unsigned long long s = 0;
            for (uint32_t w = 0; w < NT / kWave; ++w) s += red[w];
            a.counters[(size_t)qi * 8 + 3] += tot;
            a.counters[(size_t)qi * 8 + 4] += s;
        }
    }
}

hipError_t launch_refine(const RefineArgs& a, hipStream_t stream) {
    if (a.nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine, dim3(a.nq), dim3(kRefineThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace seismic_dev
