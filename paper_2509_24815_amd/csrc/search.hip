// Algorithm 2 ("Query processing with Seismic", Section 4.5) with the
// kappa-NN refinement disabled: one workgroup answers one query.
//
//   1. query ingest: membership bitmap + prefix counts + values in LDS; the
//      cut keeps the query_cut largest entries (value desc, term asc);
//   2. per cut list, in cut order:
//      a. summary scores r_j = <q, S_j> of every block (one wave per block,
//         lanes stride the block's (term, code) entries), in fp64 as
//         m * sum(q) + delta * sum(q * code), exact for values in
//         [2^-6, 2^6] because m and delta sit on the 2^-14 grid;
//      b. LDS bitonic sort of (r desc, block asc);
//      c. blocks in that order until the first one with a full heap and
//         r * heap_factor < heap.min: every document of the block is scored
//         exactly (16 lanes per document, fp64 sum of exact fp32 products)
//         and folded into the LDS top-k.
#include "device_common.h"
#include "search_kernels.h"

namespace seismic_dev {

struct SearchSmem {
    QTable q;
    uint16_t* q_term;  // [kMaxQ] 0xFFFF = dropped entry
    uint16_t* q_half;  // [kMaxQ]
    uint16_t* cut;     // [kMaxQ]
    float* r;          // [P]
    uint16_t* ord;     // [P]
    uint32_t* scratch; // [kBlock]
    uint32_t* misc;    // [8]
};

__device__ __forceinline__ uint8_t* bump(uint8_t*& p, size_t bytes) {
    uint8_t* out = p;
    p += (bytes + 15) & ~size_t(15);
    return out;
}

__global__ __launch_bounds__(kBlock) void k_search_v1(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const uint32_t qi = blockIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t nw = (ix.dim + 63u) / 64u;
    const uint32_t P = a.sort_cap;

    uint8_t* p = smem;
    QTable q;
    q.bits = (uint64_t*)bump(p, 8ull * nw);
    q.pref = (uint16_t*)bump(p, 2ull * nw);
    q.val = (float*)bump(p, 4ull * kMaxQ);
    uint16_t* q_term = (uint16_t*)bump(p, 2ull * kMaxQ);
    uint16_t* q_half = (uint16_t*)bump(p, 2ull * kMaxQ);
    uint16_t* cut = (uint16_t*)bump(p, 2ull * kMaxQ);
    float* r = (float*)bump(p, 4ull * P);
    uint16_t* ord = (uint16_t*)bump(p, 2ull * P);
    uint32_t* scratch = (uint32_t*)bump(p, 4ull * kBlock);
    uint32_t* misc = (uint32_t*)bump(p, 4ull * 8);
    TopK top;
    top.hs[0] = (float*)bump(p, 4ull * a.k);
    top.hs[1] = (float*)bump(p, 4ull * a.k);
    top.hid[0] = (uint32_t*)bump(p, 4ull * a.k);
    top.hid[1] = (uint32_t*)bump(p, 4ull * a.k);
    top.cs = (float*)bump(p, 4ull * 2 * kBlock);
    top.cid = (uint32_t*)bump(p, 4ull * 2 * kBlock);
    top.flag = (uint32_t*)bump(p, 4ull * (kBlock + 32));
    top.cur = 0;
    top.hn = 0;
    top.k = a.k;

    // ---------------------------------------------------------- ingest
    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    const uint64_t raw = q1 - q0;
    const uint32_t nqe = (uint32_t)min<uint64_t>(raw, (uint64_t)kMaxQ);
    for (uint32_t i = tid; i < nw; i += kBlock) q.bits[i] = 0ull;
    if (tid < 8) misc[tid] = 0;
    __syncthreads();
    uint32_t st = (raw > (uint64_t)kMaxQ) ? 4u : 0u;
    for (uint32_t j = tid; j < nqe; j += kBlock) {
        const uint32_t w = a.q_words[q0 + j];
        const uint32_t t = w & 0xFFFFu, h = w >> 16;
        bool keep = true;
        if (t >= ix.dim) { st |= 1u; keep = false; }
        if (!half_ok(h)) { st |= 8u; keep = false; }
        if (j > 0 && t <= (a.q_words[q0 + j - 1] & 0xFFFFu)) st |= 2u;
        if (keep) {
            const uint64_t bit = 1ull << (t & 63u);
            const uint64_t old = atomicOr((unsigned long long*)&q.bits[t >> 6], (unsigned long long)bit);
            if (old & bit) { st |= 2u; keep = false; }  // repeated term: first writer wins
        }
        q_term[j] = keep ? (uint16_t)t : (uint16_t)0xFFFFu;
        q_half[j] = (uint16_t)h;
    }
    if (st) atomicOr(&misc[0], st);
    __syncthreads();
    build_prefix(q.bits, q.pref, nw, scratch);
    uint32_t nvalid_local = 0;
    for (uint32_t j = tid; j < nqe; j += kBlock) {
        const uint32_t t = q_term[j];
        if (t == 0xFFFFu) continue;
        const uint64_t w = q.bits[t >> 6];
        const uint32_t slot = q.pref[t >> 6] + (uint32_t)__popcll(w & ((1ull << (t & 63u)) - 1ull));
        q.val[slot] = half_bits_to_float(q_half[j]);
        ++nvalid_local;
    }
    if (nvalid_local) atomicAdd(&misc[1], nvalid_local);
    __syncthreads();
    const uint32_t nvalid = misc[1];
    const uint32_t ncut = (a.cut == 0 || a.cut > nvalid) ? nvalid : a.cut;
    // cut order: value desc (positive fp16: bit order), then term asc
    for (uint32_t j = tid; j < nqe; j += kBlock) {
        const uint32_t t = q_term[j];
        if (t == 0xFFFFu) continue;
        const uint32_t h = q_half[j];
        uint32_t rank = 0;
        for (uint32_t i = 0; i < nqe; ++i) {
            const uint32_t ti = q_term[i];
            if (ti == 0xFFFFu) continue;
            const uint32_t hi = q_half[i];
            rank += (hi > h || (hi == h && ti < t)) ? 1u : 0u;
        }
        if (rank < ncut) cut[rank] = (uint16_t)t;
    }
    __syncthreads();

    // counters (thread 0 keeps the uniform ones)
    uint64_t c_sum = 0, c_blocks = 0, c_eval = 0, c_docs = 0, c_tests = 0;
    uint64_t c_nnz = 0;  // per thread, reduced at the end

    for (uint32_t ci = 0; ci < ncut; ++ci) {
        const uint32_t t = cut[ci];
        const uint32_t b0 = ix.list_off[t], b1 = ix.list_off[t + 1];
        const uint32_t nb = b1 - b0;
        if (nb == 0) {
            if (a.prefix && tid == 0 && ci < a.prefix_stride) a.prefix[(size_t)qi * a.prefix_stride + ci] = 0;
            continue;
        }
        c_sum += ix.blk_sum_off[b1] - ix.blk_sum_off[b0];
        c_blocks += nb;
        // ------------------------------------------ a. summary scores
        for (uint32_t bl = wave; bl < nb; bl += kBlock / kWave) {
            const uint32_t b = b0 + bl;
            const uint64_t s0 = ix.blk_sum_off[b], s1 = ix.blk_sum_off[b + 1];
            double A = 0.0, B = 0.0;
            for (uint64_t e = s0 + lane; e < s1; e += kWave) {
                float qv;
                if (q_lookup(q, ix.sum_term[e], qv)) {
                    A += (double)qv;
                    B += (double)(qv * (float)ix.sum_code[e]);  // exact: 11 x 8 bits
                }
            }
            A = wave_sum(A);
            B = wave_sum(B);
            if (lane == 0) r[bl] = (float)((double)ix.blk_m[b] * A + (double)ix.blk_delta[b] * B);
        }
        uint32_t Pl = 2;
        while (Pl < nb) Pl <<= 1;
        for (uint32_t i = tid; i < Pl; i += kBlock) {
            if (i >= nb) r[i] = -INFINITY;
            ord[i] = (uint16_t)i;
        }
        __syncthreads();
        // ------------------------------------------ b. bitonic sort
        for (uint32_t kk = 2; kk <= Pl; kk <<= 1) {
            for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < Pl; i += kBlock) {
                    const uint32_t l = i ^ j;
                    if (l > i) {
                        const float ri = r[i], rl = r[l];
                        const uint32_t oi = ord[i], ol = ord[l];
                        const bool l_first = rl > ri || (rl == ri && ol < oi);
                        const bool up = (i & kk) == 0;
                        if (up ? l_first : !l_first) {
                            r[i] = rl; r[l] = ri; ord[i] = (uint16_t)ol; ord[l] = (uint16_t)oi;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // ------------------------------------------ c. traversal
        uint32_t pos = 0;
        for (; pos < nb; ++pos) {
            const float rj = r[pos];
            if (ord[pos] >= nb) break;  // only padding left (cannot happen for finite scores)
            const uint32_t b = b0 + ord[pos];
            if (top.hn == top.k) {
                ++c_tests;
                if ((double)rj * (double)a.hf < (double)top.hs[top.cur][top.k - 1]) break;
            }
            const uint32_t p0 = ix.blk_post_off[b], p1 = ix.blk_post_off[b + 1];
            ++c_eval;
            c_docs += p1 - p0;
            for (uint32_t c0 = p0; c0 < p1; c0 += kBlock / 16) {
                const uint32_t g = tid >> 4, gl = tid & 15u;
                const uint32_t pp = c0 + g;
                double acc = 0.0;
                uint32_t d = 0;
                if (pp < p1) {
                    d = ix.postings[pp];
                    const uint64_t rs = ix.row_ptr[d], re = ix.row_ptr[d + 1];
                    if (gl == 0) c_nnz += re - rs;
                    for (uint64_t e = rs + gl; e < re; e += 16) {
                        const uint32_t w = ix.words[e];
                        float qv;
                        if (q_lookup(q, w & 0xFFFFu, qv)) acc += (double)(qv * half_bits_to_float(w >> 16));
                    }
                }
                acc = group_sum<double, 16>(acc);
                if (gl == 0 && pp < p1) { top.cs[g] = (float)acc; top.cid[g] = d; }
                __syncthreads();
                top.merge(min(p1 - c0, (uint32_t)(kBlock / 16)));
            }
        }
        if (a.prefix && tid == 0 && ci < a.prefix_stride)
            a.prefix[(size_t)qi * a.prefix_stride + ci] = (uint16_t)min(pos, 65535u);
        __syncthreads();  // r/ord are rewritten by the next list
    }

    // ------------------------------------------------------------ output
    for (uint32_t i = tid; i < a.k; i += kBlock) {
        const bool have = i < top.hn;
        a.out_ids[(size_t)qi * a.k + i] = have ? top.hid[top.cur][i] : 0xFFFFFFFFu;
        a.out_scores[(size_t)qi * a.k + i] = have ? top.hs[top.cur][i] : -INFINITY;
    }
    if (a.prefix)
        for (uint32_t i = ncut + tid; i < a.prefix_stride; i += kBlock) a.prefix[(size_t)qi * a.prefix_stride + i] = 0;
    if (a.counters) {
        // block reduction of c_nnz
        unsigned long long v = wave_sum((unsigned long long)c_nnz);
        __syncthreads();
        if (lane == 0) ((unsigned long long*)scratch)[wave] = v;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < kBlock / kWave; ++w) tot += ((unsigned long long*)scratch)[w];
            uint64_t* c = a.counters + (size_t)qi * 8;
            c[0] = c_sum; c[1] = c_blocks; c[2] = c_eval; c[3] = c_docs; c[4] = tot; c[5] = c_tests;
            c[6] = misc[0]; c[7] = ncut;
        }
    }
}

size_t search_v1_smem_bytes(uint32_t dim, uint32_t sort_cap, uint32_t k) {
    auto r16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    size_t nw = (dim + 63) / 64;
    size_t s = 0;
    s += r16(8 * nw) + r16(2 * nw) + r16(4 * kMaxQ) + 3 * r16(2 * kMaxQ);
    s += r16(4 * (size_t)sort_cap) + r16(2 * (size_t)sort_cap) + r16(4 * kBlock) + r16(32);
    s += 4 * r16(4 * (size_t)k) + 2 * r16(4 * 2 * kBlock) + r16(4 * (kBlock + 32));
    return s;
}

hipError_t launch_search_v1(const SearchArgs& a, uint32_t nq, size_t smem, hipStream_t stream) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_search_v1, dim3(nq), dim3(kBlock), smem, stream, a);
    return hipGetLastError();
}

}  // namespace seismic_dev
