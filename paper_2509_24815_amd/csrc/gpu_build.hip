// Index build on the GPU (Algorithm "Indexing with Seismic", Section 4.4),
// producing byte for byte the index the host builder produces.
//
// The device transposes the forward index (column lists, doc ascending;
// csc.hip), the host decides per term the kept count n = min(|L_i|, cap_i)
// and the block count nb; everything else runs in one kernel, a workgroup
// per term pulled from a queue (longest lists first), launched over slices
// of that order:
//   A. Set alpha-MSS: the n largest values of the column (value desc, doc
//      asc) found by a two-level histogram over the fp16 bits, then a
//      stream compaction in column order (so the kept list stays doc
//      ascending, as the host stores it);
//   B. centroid sampling: the host's SplitMix64 partial Fisher-Yates, run by
//      one thread;
//   C. shallow K-means assignment (Section 4.1.2): the centroids' rows become
//      a term -> (centroid, value) table; a wave per document accumulates
//      exact fp64 inner products with every centroid in LDS and takes the
//      argmax (lowest centroid on ties);
//   D. blocks in centroid order, empty ones dropped, documents ascending;
//   E. per block, the max vector phi over the block's rows, its gamma-MSS
//      (value desc, term asc; the boundary found by two histograms of exact
//      integer masses) and the u8 quantization on the 2^-14 grid.
// Summaries go to a bump-allocated region.  seismic_build_index_gpu
// assembles the final arrays in canonical order on the host;
// seismic_build_index_device gathers them on the device and leaves the
// index there.  A term beyond the kernel's capacities makes either report
// EINVAL (the host builder has no such limits).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "device_internal.h"

using namespace seismic;

namespace seismic_dev {

namespace {

constexpr uint32_t kBT = 256;            // threads per workgroup
constexpr uint32_t kBWaves = kBT / kWave;
constexpr uint32_t kMaxNb = 1024;        // blocks per list handled on the GPU
constexpr uint32_t kLdsSort = 4096;      // entries sorted in LDS; longer runs use global scratch

struct BuildArgs {
    const uint64_t* row_ptr;
    const uint32_t* words;
    uint32_t dim;
    const uint64_t* csc_off;
    const uint32_t* csc_doc;
    const uint16_t* csc_val;
    const uint32_t* order;  // terms with n > 0, longest first
    uint32_t n_work;
    const uint32_t* t_n;
    const uint32_t* t_nb;
    const uint64_t* t_post;  // posting offset of each term
    const uint64_t* t_bcap;  // block-slot offset of each term (nb slots)
    uint32_t* queue;
    uint64_t seed;
    double gamma;
    // outputs
    uint32_t* list_docs;  // kept lists, doc ascending
    uint32_t* postings;   // block order
    uint32_t* t_nblk;
    uint32_t* b_len;
    uint32_t* b_cent;
    float* b_m;
    float* b_delta;
    uint64_t* b_sum_at;
    uint32_t* b_sum_len;
    uint16_t* sum_term;
    uint8_t* sum_code;
    unsigned long long* sum_bump;
    uint64_t sum_cap;
    uint32_t* flags;  // 4: summary region, 8: centroid table
    // per-workgroup scratch
    uint32_t* s_perm;
    uint32_t* s_assign;
    uint64_t s_ncap;
    uint32_t* s_tcount;  // dim each (zero between terms)
    uint32_t* s_tstart;
    uint32_t* s_tfill;
    uint32_t* s_touched;
    uint32_t* s_phi;
    uint16_t* s_ck;
    uint16_t* s_cv;
    uint64_t s_ecap;
    uint32_t* s_sort;    // next power of two >= dim each
    uint32_t s_sortcap;
};

struct BuildLds {
    uint32_t cnt1[256];
    unsigned long long mass1[256];
    uint32_t cnt2[128];
    unsigned long long mass2[128];
    uint32_t cent[kMaxNb];
    uint32_t cntk[kMaxNb];
    uint32_t startk[kMaxNb];
    uint32_t lbk[kMaxNb];
    double acc[kBWaves][kMaxNb];
    uint32_t buf[kLdsSort];  // ties, then kept terms (short runs)
    uint32_t scratch[kBWaves + 1];
    uint32_t misc[16];
    unsigned long long umisc[8];
};

__device__ __forceinline__ uint64_t units24(uint32_t h) {
    const uint32_t e = (h >> 10) & 0x1Fu;
    const uint64_t f = h & 0x3FFu;
    return e == 0 ? f : ((1024ull + f) << (e - 1));
}

__device__ __forceinline__ double mass_of(unsigned long long u) { return ldexp((double)u, -24); }

// SplitMix64 step and bounded draw (128-bit product), as the host builder.
__device__ __forceinline__ uint64_t splitmix_next(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Ascending bitonic sort of a[0, n) (LDS, or the workgroup's global
// scratch for long arrays; capacity >= the next power of two), padding
// with ~0.
__device__ void wg_sort(uint32_t* a, uint32_t n) {
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t i = n + threadIdx.x; i < P; i += kBT) a[i] = 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kBT) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t x = a[i], y = a[l];
                    if (((i & k) == 0) ? (x > y) : (x < y)) { a[i] = y; a[l] = x; }
                }
            }
            __syncthreads();
        }
}

// Block-wide exclusive scan (all threads call).
__device__ __forceinline__ uint32_t bscan(uint32_t v, uint32_t* scratch, uint32_t* total) {
    return block_exscan<(int)kBT>(v, scratch, total);
}

}  // namespace

__global__ __launch_bounds__(kBT) void k_build_terms(BuildArgs a) {
    __shared__ BuildLds L;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t* perm = a.s_perm + (size_t)blockIdx.x * a.s_ncap;
    uint32_t* assign = a.s_assign + (size_t)blockIdx.x * a.s_ncap;
    uint32_t* tcount = a.s_tcount + (size_t)blockIdx.x * a.dim;
    uint32_t* tstart = a.s_tstart + (size_t)blockIdx.x * a.dim;
    uint32_t* tfill = a.s_tfill + (size_t)blockIdx.x * a.dim;
    uint32_t* touched = a.s_touched + (size_t)blockIdx.x * a.dim;
    uint32_t* phi = a.s_phi + (size_t)blockIdx.x * a.dim;
    uint16_t* ck = a.s_ck + (size_t)blockIdx.x * a.s_ecap;
    uint16_t* cv = a.s_cv + (size_t)blockIdx.x * a.s_ecap;
    uint32_t* gsort = a.s_sort + (size_t)blockIdx.x * a.s_sortcap;

    for (;;) {
        if (tid == 0) L.misc[0] = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t w = L.misc[0];
        __syncthreads();
        if (w >= a.n_work) break;
        const uint32_t t = a.order[w];
        const uint32_t n = a.t_n[t], nb = a.t_nb[t];
        const uint64_t po = a.t_post[t], bo = a.t_bcap[t];
        const uint64_t c0 = a.csc_off[t], nf = a.csc_off[t + 1] - c0;
        uint32_t* list = a.list_docs + po;

        // ------------------------------------------------ A. Set alpha-MSS
        if (nf <= n) {
            for (uint32_t i = tid; i < n; i += kBT) list[i] = a.csc_doc[c0 + i];
        } else {
            for (uint32_t i = tid; i < 256; i += kBT) L.cnt1[i] = 0;
            if (tid < 128) L.cnt2[tid] = 0;
            __syncthreads();
            for (uint64_t i = tid; i < nf; i += kBT) atomicAdd(&L.cnt1[a.csc_val[c0 + i] >> 7], 1u);
            __syncthreads();
            if (tid == 0) {
                uint32_t above = 0, b = 255;
                for (;; --b) {
                    if (above + L.cnt1[b] >= n || b == 0) break;
                    above += L.cnt1[b];
                }
                L.misc[1] = b;
                L.misc[2] = above;
            }
            __syncthreads();
            const uint32_t B1 = L.misc[1];
            for (uint64_t i = tid; i < nf; i += kBT) {
                const uint32_t h = a.csc_val[c0 + i];
                if ((h >> 7) == B1) atomicAdd(&L.cnt2[h & 127u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t above = L.misc[2], b = 127;
                for (;; --b) {
                    if (above + L.cnt2[b] >= n || b == 0) break;
                    above += L.cnt2[b];
                }
                L.misc[3] = (B1 << 7) | b;  // boundary value
                L.misc[4] = n - above;      // entries of that value to keep, smallest doc ids first
            }
            __syncthreads();
            const uint32_t vstar = L.misc[3], r = L.misc[4];
            uint32_t eq_before = 0, kept_before = 0;
            for (uint64_t base = 0; base < nf; base += kBT) {
                const uint64_t i = base + tid;
                uint32_t h = 0;
                if (i < nf) h = a.csc_val[c0 + i];
                const bool eq = i < nf && h == vstar;
                uint32_t eq_tot;
                const uint32_t eq_rank = eq_before + bscan(eq ? 1u : 0u, L.scratch, &eq_tot);
                const bool keep = i < nf && (h > vstar || (eq && eq_rank < r));
                uint32_t k_tot;
                const uint32_t at = kept_before + bscan(keep ? 1u : 0u, L.scratch, &k_tot);
                if (keep && at < n) list[at] = a.csc_doc[c0 + i];
                eq_before += eq_tot;
                kept_before += k_tot;
            }
        }
        __syncthreads();

        // --------------------------------------------- B. centroid sampling
        for (uint32_t i = tid; i < n; i += kBT) perm[i] = i;
        __syncthreads();
        if (tid == 0) {
            uint64_t s = a.seed ^ (0xD1B54A32D192ED03ull * ((uint64_t)t + 1));
            for (uint32_t i = 0; i < nb; ++i) {
                const uint64_t z = splitmix_next(s);
                const uint32_t j = i + (uint32_t)__umul64hi(z, (uint64_t)(n - i));
                const uint32_t x = perm[i];
                perm[i] = perm[j];
                perm[j] = x;
            }
        }
        __syncthreads();
        for (uint32_t k = tid; k < nb; k += kBT) L.cent[k] = list[perm[k]];
        __syncthreads();

        // ----------------------------------------------- C. assignment
        if (nb > 1) {
            if (tid == 0) { L.misc[5] = 0; L.misc[6] = 0; }
            __syncthreads();
            // count centroid entries per term; remember each touched term once
            for (uint32_t k = wave; k < nb; k += kBWaves) {
                const uint32_t d = L.cent[k];
                const uint64_t r0 = a.row_ptr[d], r1 = a.row_ptr[d + 1];
                for (uint64_t j = r0 + lane; j < r1; j += kWave) {
                    const uint32_t term = a.words[j] & 0xFFFFu;
                    if (atomicAdd(&tcount[term], 1u) == 0u) touched[atomicAdd(&L.misc[5], 1u)] = term;
                }
            }
            __syncthreads();
            const uint32_t nt = L.misc[5];
            uint32_t run = 0;
            for (uint32_t base = 0; base < nt; base += kBT) {
                const uint32_t u = base + tid;
                const uint32_t c = u < nt ? tcount[touched[u]] : 0u;
                uint32_t tot;
                const uint32_t at = run + bscan(c, L.scratch, &tot);
                if (u < nt) tstart[touched[u]] = at;
                run += tot;
            }
            if (run > a.s_ecap) {
                // the host discards this index build; keep the later steps in bounds
                if (tid == 0) atomicOr(a.flags, 8u);
                for (uint32_t i = tid; i < n; i += kBT) assign[i] = 0;
            } else {
                __syncthreads();
                for (uint32_t k = wave; k < nb; k += kBWaves) {
                    const uint32_t d = L.cent[k];
                    const uint64_t r0 = a.row_ptr[d], r1 = a.row_ptr[d + 1];
                    for (uint64_t j = r0 + lane; j < r1; j += kWave) {
                        const uint32_t wd = a.words[j];
                        const uint32_t term = wd & 0xFFFFu;
                        const uint32_t pos = tstart[term] + atomicAdd(&tfill[term], 1u);
                        ck[pos] = (uint16_t)k;
                        cv[pos] = (uint16_t)(wd >> 16);
                    }
                }
                __syncthreads();
                double* acc = L.acc[wave];
                for (uint32_t k = lane; k < nb; k += kWave) acc[k] = 0.0;
                for (uint32_t i = wave; i < n; i += kBWaves) {
                    const uint32_t d = list[i];
                    const uint64_t r0 = a.row_ptr[d], r1 = a.row_ptr[d + 1];
                    for (uint64_t j = r0; j < r1; ++j) {
                        const uint32_t wd = a.words[j];
                        const uint32_t term = wd & 0xFFFFu;
                        const uint32_t c = tcount[term];
                        if (c == 0) continue;
                        const double vd = (double)half_bits_to_float(wd >> 16);
                        const uint32_t s0 = tstart[term];
                        // centroids holding this term are distinct: no two lanes share a k
                        for (uint32_t e = lane; e < c; e += kWave)
                            acc[ck[s0 + e]] += vd * (double)half_bits_to_float(cv[s0 + e]);
                    }
                    // argmax, lowest centroid on ties
                    double bv = -1.0;
                    uint32_t bk = 0xFFFFFFFFu;
                    for (uint32_t k = lane; k < nb; k += kWave) {
                        const double v = acc[k];
                        if (bk == 0xFFFFFFFFu || v > bv) { bv = v; bk = k; }
                        acc[k] = 0.0;
                    }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        const double ov = __shfl_xor(bv, o, kWave);
                        const uint32_t ok = __shfl_xor(bk, o, kWave);
                        if (ok != 0xFFFFFFFFu && (bk == 0xFFFFFFFFu || ov > bv || (ov == bv && ok < bk))) {
                            bv = ov;
                            bk = ok;
                        }
                    }
                    if (lane == 0) assign[i] = bk;
                }
            }
            __syncthreads();
            for (uint32_t u = tid; u < nt; u += kBT) {
                tcount[touched[u]] = 0u;
                tfill[touched[u]] = 0u;
            }
        } else {
            for (uint32_t i = tid; i < n; i += kBT) assign[i] = 0;
        }
        __syncthreads();

        // --------------------------------------------------- D. blocks
        for (uint32_t k = tid; k < nb; k += kBT) L.cntk[k] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kBT) atomicAdd(&L.cntk[min(assign[i], nb - 1)], 1u);
        __syncthreads();
        {
            uint32_t run_p = 0, run_b = 0;
            for (uint32_t base = 0; base < nb; base += kBT) {
                const uint32_t k = base + tid;
                const uint32_t c = k < nb ? L.cntk[k] : 0u;
                uint32_t tp, tb;
                const uint32_t sp = run_p + bscan(c, L.scratch, &tp);
                const uint32_t sb = run_b + bscan(c ? 1u : 0u, L.scratch, &tb);
                if (k < nb) { L.startk[k] = sp; L.lbk[k] = c ? sb : 0xFFFFFFFFu; }
                run_p += tp;
                run_b += tb;
            }
            if (tid == 0) a.t_nblk[t] = run_b;
        }
        __syncthreads();
        for (uint32_t k = tid; k < nb; k += kBT) {
            const uint32_t c = L.cntk[k];
            if (!c) continue;
            uint32_t* out = a.postings + po + L.startk[k];
            uint32_t m = 0;
            for (uint32_t i = 0; i < n && m < c; ++i)
                if (min(assign[i], nb - 1) == k) out[m++] = list[i];
            const uint64_t b = bo + L.lbk[k];
            a.b_len[b] = c;
            a.b_cent[b] = L.cent[k];
        }
        __syncthreads();

        // ------------------------------------------------- E. summaries
        for (uint32_t k = 0; k < nb; ++k) {
            const uint32_t c = L.cntk[k];
            if (!c) continue;
            const uint32_t* docs = a.postings + po + L.startk[k];
            const uint64_t b = bo + L.lbk[k];
            if (tid == 0) { L.misc[7] = 0; L.umisc[0] = 0; L.umisc[1] = ~0ull; L.umisc[2] = 0; }
            for (uint32_t i = tid; i < 256; i += kBT) { L.cnt1[i] = 0; L.mass1[i] = 0; }
            if (tid < 128) { L.cnt2[tid] = 0; L.mass2[tid] = 0; }
            __syncthreads();
            // phi = max over the block's rows (positive fp16: bit order is value order)
            for (uint32_t q = wave; q < c; q += kBWaves) {
                const uint32_t d = docs[q];
                const uint64_t r0 = a.row_ptr[d], r1 = a.row_ptr[d + 1];
                for (uint64_t j = r0 + lane; j < r1; j += kWave) {
                    const uint32_t wd = a.words[j];
                    const uint32_t term = wd & 0xFFFFu;
                    if (atomicMax(&phi[term], wd >> 16) == 0u) touched[atomicAdd(&L.misc[7], 1u)] = term;
                }
            }
            __syncthreads();
            const uint32_t nt = L.misc[7];
            for (uint32_t u = tid; u < nt; u += kBT) {
                const uint32_t h = phi[touched[u]];
                const unsigned long long m = units24(h);
                atomicAdd(&L.umisc[0], m);
                atomicAdd(&L.cnt1[h >> 7], 1u);
                atomicAdd(&L.mass1[h >> 7], m);
            }
            __syncthreads();
            const double need = a.gamma * mass_of(L.umisc[0]);
            if (tid == 0) {
                unsigned long long cum = 0;
                uint32_t bb = 255;
                for (;; --bb) {
                    if (mass_of(cum + L.mass1[bb]) >= need || bb == 0) break;
                    cum += L.mass1[bb];
                }
                L.misc[8] = bb;
                L.umisc[3] = cum;
            }
            __syncthreads();
            const uint32_t B1 = L.misc[8];
            for (uint32_t u = tid; u < nt; u += kBT) {
                const uint32_t h = phi[touched[u]];
                if ((h >> 7) == B1) { atomicAdd(&L.cnt2[h & 127u], 1u); atomicAdd(&L.mass2[h & 127u], units24(h)); }
            }
            __syncthreads();
            if (tid == 0) {
                unsigned long long cum = L.umisc[3];
                uint32_t bb = 127;
                for (;; --bb) {
                    if (mass_of(cum + L.mass2[bb]) >= need || bb == 0) break;
                    cum += L.mass2[bb];
                }
                L.misc[9] = (B1 << 7) | bb;  // boundary value
                L.umisc[4] = cum;            // mass of the larger values
                L.misc[10] = 0;              // ties collected
            }
            __syncthreads();
            const uint32_t vstar = L.misc[9];
            // entries with the boundary value, term ascending, are taken until the mass suffices
            uint32_t nties = 0;
            for (uint32_t u = tid; u < nt; u += kBT) nties += phi[touched[u]] == vstar ? 1u : 0u;
            uint32_t tot_ties;
            (void)bscan(nties, L.scratch, &tot_ties);
            uint32_t* tb = tot_ties <= kLdsSort ? L.buf : gsort;
            for (uint32_t u = tid; u < nt; u += kBT) {
                const uint32_t term = touched[u];
                if (phi[term] == vstar) tb[atomicAdd(&L.misc[10], 1u)] = term;
            }
            __syncthreads();
            wg_sort(tb, tot_ties);
            if (tid == 0) {
                unsigned long long cum = L.umisc[4];
                const unsigned long long uv = units24(vstar);
                uint32_t r = 0;
                while (r < tot_ties) {
                    cum += uv;
                    ++r;
                    if (mass_of(cum) >= need) break;
                }
                L.misc[11] = r;
                L.misc[12] = 0;
                L.misc[13] = tb[r ? r - 1 : 0];  // largest tied term kept
            }
            __syncthreads();
            const uint32_t r = L.misc[11], tie_last = L.misc[13];
            // kept: larger values, and ties up to the r-th term
            uint32_t nkeep = 0;
            for (uint32_t u = tid; u < nt; u += kBT) {
                const uint32_t h = phi[touched[u]];
                nkeep += (h > vstar || (h == vstar && r > 0 && touched[u] <= tie_last)) ? 1u : 0u;
            }
            uint32_t nk;
            (void)bscan(nkeep, L.scratch, &nk);
            uint32_t* kb = nk <= kLdsSort ? L.buf : gsort;
            for (uint32_t u = tid; u < nt; u += kBT) {
                const uint32_t term = touched[u];
                const uint32_t h = phi[term];
                if (h > vstar || (h == vstar && r > 0 && term <= tie_last)) {
                    kb[atomicAdd(&L.misc[12], 1u)] = term;
                    const unsigned long long m = units24(h);
                    atomicMin(&L.umisc[1], m);
                    atomicMax(&L.umisc[2], m);
                }
            }
            __syncthreads();
            wg_sort(kb, nk);
            if (tid == 0) L.umisc[5] = atomicAdd(a.sum_bump, (unsigned long long)nk);
            __syncthreads();
            const uint64_t at0 = L.umisc[5];
            if (at0 + nk > a.sum_cap) {
                if (tid == 0) atomicOr(a.flags, 4u);
            } else {
                const uint64_t grid = 1ull << (24 - kGridBits);
                const uint64_t m_u = (L.umisc[1] / grid) * grid;
                const uint64_t span = L.umisc[2] - m_u;
                const uint64_t d_u = ((span + 256 * grid - 1) / (256 * grid)) * grid;
                for (uint32_t j = tid; j < nk; j += kBT) {
                    const uint32_t term = kb[j];
                    const uint64_t cc = d_u ? (units24(phi[term]) - m_u) / d_u : 0;
                    a.sum_term[at0 + j] = (uint16_t)term;
                    a.sum_code[at0 + j] = (uint8_t)(cc < 255 ? cc : 255);
                }
                if (tid == 0) {
                    a.b_m[b] = (float)ldexp((double)m_u, -24);
                    a.b_delta[b] = (float)ldexp((double)d_u, -24);
                    a.b_sum_at[b] = at0;
                    a.b_sum_len[b] = nk;
                }
            }
            __syncthreads();
            for (uint32_t u = tid; u < nt; u += kBT) phi[touched[u]] = 0u;
            __syncthreads();
        }
    }
}

}  // namespace seismic_dev

// ------------------------------------------------------------ host driver

namespace {

using seismic_dev::BuildArgs;
using seismic_dev::DevCsc;
using seismic_dev::kWave;

template <typename T>
int dalloc(std::vector<void*>& keep, T*& p, size_t n) {
    p = nullptr;
    if (hipMalloc((void**)&p, std::max<size_t>(n * sizeof(T), 16)) != hipSuccess)
        return fail(SEISMIC_ENOMEM, "gpu build: device allocation of %zu bytes failed", n * sizeof(T));
    keep.push_back(p);
    return SEISMIC_OK;
}

template <typename T>
int dupload(std::vector<void*>& keep, T*& p, const T* src, size_t n) {
    int rc = dalloc(keep, p, n);
    if (rc) return rc;
    if (n && hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(SEISMIC_EHIP, "gpu build: upload failed");
    return SEISMIC_OK;
}

// Device buffers of one build; freed at scope exit unless taken.
struct Frees {
    std::vector<void*> p;
    void drop(void* x) {
        auto it = std::find(p.begin(), p.end(), x);
        if (it != p.end()) { (void)hipFree(x); p.erase(it); }
    }
    void take(void* x) {
        auto it = std::find(p.begin(), p.end(), x);
        if (it != p.end()) p.erase(it);
    }
    ~Frees() {
        for (void* x : p) (void)hipFree(x);
    }
};

// Per-term plan from the full list lengths: kept count (the list cap of
// Set alpha-MSS), block count (proportional to the kept count, at least
// one), offsets of the term's postings and block slots, and the work order
// (longest lists first).
struct Plan {
    std::vector<uint32_t> t_n, t_nb, order;
    std::vector<uint64_t> t_post, t_bcap;
    uint32_t n_max = 1, nb_max = 1;
    uint64_t total_n = 0, total_b = 0;
};

void plan_terms(const std::vector<uint64_t>& off, uint32_t dim, const seismic_build_params* p, Plan& P) {
    P.t_n.assign(dim, 0);
    P.t_nb.assign(dim, 0);
    P.t_post.assign(dim + 1, 0);
    P.t_bcap.assign(dim + 1, 0);
    P.order.clear();
    for (uint32_t t = 0; t < dim; ++t) {
        const uint64_t nf = off[t + 1] - off[t];
        uint64_t n = std::min<uint64_t>(nf, list_cap(nf, p->lambda, p->alpha));
        uint64_t nb = 0;
        if (n) {
            nb = ((uint64_t)p->beta * n + p->lambda - 1) / p->lambda;
            nb = std::max<uint64_t>(1, std::min<uint64_t>(nb, n));
            P.order.push_back(t);
        }
        P.t_n[t] = (uint32_t)std::min<uint64_t>(n, 0xFFFFFFFFull);
        P.t_nb[t] = (uint32_t)std::min<uint64_t>(nb, 0xFFFFFFFFull);
        P.t_post[t + 1] = P.t_post[t] + n;
        P.t_bcap[t + 1] = P.t_bcap[t] + nb;
        P.n_max = (uint32_t)std::max<uint64_t>(P.n_max, std::min<uint64_t>(n, 0xFFFFFFFFull));
        P.nb_max = (uint32_t)std::max<uint64_t>(P.nb_max, std::min<uint64_t>(nb, 0xFFFFFFFFull));
    }
    std::stable_sort(P.order.begin(), P.order.end(), [&](uint32_t x, uint32_t y) { return P.t_n[x] > P.t_n[y]; });
    P.total_n = P.t_post[dim];
    P.total_b = P.t_bcap[dim];
}

bool plan_fits(const Plan& P) { return P.nb_max <= seismic_dev::kMaxNb && P.n_max <= (1u << 24); }

// Runs the per-term kernel over device rows d_rp/d_w and their column lists.
// On return (SEISMIC_OK) a holds the device outputs (owned by F) and flags
// the kernel's flags (0: complete).
int run_terms(const uint64_t* d_rp, const uint32_t* d_w, uint32_t dim, uint32_t row_max, const DevCsc& csc,
              const Plan& P, const seismic_build_params* p, int device, Frees& F, BuildArgs& a, uint32_t& flags,
              uint64_t*& d_bsat) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(SEISMIC_EHIP, "gpu build: device query failed");
    const uint32_t grid = (uint32_t)std::max(1, prop.multiProcessorCount) * 2;
    const uint64_t ecap = (uint64_t)P.nb_max * std::max<uint32_t>(row_max, 1);
    uint32_t *d_order = nullptr, *d_tn = nullptr, *d_tnb = nullptr, *d_q = nullptr;
    uint64_t *d_tpost = nullptr, *d_tbcap = nullptr;
    a = BuildArgs{};
    int rc = SEISMIC_OK;
    if (!rc) rc = dupload(F.p, d_order, P.order.data(), P.order.size());
    if (!rc) rc = dupload(F.p, d_tn, P.t_n.data(), P.t_n.size());
    if (!rc) rc = dupload(F.p, d_tnb, P.t_nb.data(), P.t_nb.size());
    if (!rc) rc = dupload(F.p, d_tpost, P.t_post.data(), P.t_post.size());
    if (!rc) rc = dupload(F.p, d_tbcap, P.t_bcap.data(), P.t_bcap.size());
    if (!rc) rc = dalloc(F.p, d_q, 4);
    a.row_ptr = d_rp; a.words = d_w; a.dim = dim; a.csc_off = csc.off; a.csc_doc = csc.doc; a.csc_val = csc.val;
    a.order = d_order; a.n_work = (uint32_t)P.order.size(); a.t_n = d_tn; a.t_nb = d_tnb; a.t_post = d_tpost;
    a.t_bcap = d_tbcap; a.queue = d_q; a.seed = p->seed; a.gamma = p->gamma;
    const uint64_t total_n = P.total_n, total_b = P.total_b;
    if (!rc) rc = dalloc(F.p, a.list_docs, total_n);
    if (!rc) rc = dalloc(F.p, a.postings, total_n);
    if (!rc) rc = dalloc(F.p, a.t_nblk, dim);
    if (!rc) rc = dalloc(F.p, a.b_len, total_b);
    if (!rc) rc = dalloc(F.p, a.b_cent, total_b);
    if (!rc) rc = dalloc(F.p, a.b_m, total_b);
    if (!rc) rc = dalloc(F.p, a.b_delta, total_b);
    if (!rc) rc = dalloc(F.p, d_bsat, total_b);
    a.b_sum_at = d_bsat;
    if (!rc) rc = dalloc(F.p, a.b_sum_len, total_b);
    if (!rc) rc = dalloc(F.p, a.sum_bump, 1);
    if (!rc) rc = dalloc(F.p, a.flags, 1);
    a.s_ncap = P.n_max;
    a.s_ecap = ecap;
    if (!rc) rc = dalloc(F.p, a.s_perm, (size_t)grid * P.n_max);
    if (!rc) rc = dalloc(F.p, a.s_assign, (size_t)grid * P.n_max);
    if (!rc) rc = dalloc(F.p, a.s_tcount, (size_t)grid * dim);
    if (!rc) rc = dalloc(F.p, a.s_tstart, (size_t)grid * dim);
    if (!rc) rc = dalloc(F.p, a.s_tfill, (size_t)grid * dim);
    if (!rc) rc = dalloc(F.p, a.s_touched, (size_t)grid * dim);
    if (!rc) rc = dalloc(F.p, a.s_phi, (size_t)grid * dim);
    if (!rc) rc = dalloc(F.p, a.s_ck, (size_t)grid * ecap);
    if (!rc) rc = dalloc(F.p, a.s_cv, (size_t)grid * ecap);
    uint32_t sortcap = 1;
    while (sortcap < dim) sortcap <<= 1;
    a.s_sortcap = sortcap;
    if (!rc) rc = dalloc(F.p, a.s_sort, (size_t)grid * sortcap);
    if (rc) return rc;
    // the summary region, sized last: room for 1024 entries per block where
    // the free memory allows (at least 256; the kernel reports the exact
    // need when the region is short, and the slices then run again)
    {
        size_t free_b = 0, total_mem = 0;
        (void)hipMemGetInfo(&free_b, &total_mem);
        const uint64_t lo = std::max<uint64_t>(P.total_b * 256, 1 << 20);
        const uint64_t room = free_b > (4ull << 30) ? (free_b - (4ull << 30)) / 3 : 0;
        a.sum_cap = std::max(lo, std::min<uint64_t>(P.total_b * 1024, room));
    }
    if (!rc) rc = dalloc(F.p, a.sum_term, a.sum_cap);
    if (!rc) rc = dalloc(F.p, a.sum_code, a.sum_cap);
    if (rc) return rc;
    bool ok = hipMemset(d_q, 0, 4) == hipSuccess && hipMemset(a.sum_bump, 0, 8) == hipSuccess &&
              hipMemset(a.t_nblk, 0, (size_t)dim * 4) == hipSuccess &&
              hipMemset(a.flags, 0, 4) == hipSuccess &&
              hipMemset(a.s_tcount, 0, (size_t)grid * dim * 4) == hipSuccess &&
              hipMemset(a.s_tfill, 0, (size_t)grid * dim * 4) == hipSuccess &&
              hipMemset(a.s_phi, 0, (size_t)grid * dim * 4) == hipSuccess;
    if (!ok) return fail(SEISMIC_EHIP, "gpu build: memset failed");
    // launches over slices of the work order of about equal cost (kept
    // postings times blocks, the assignment's size), so that a long build
    // reports progress between launches
    std::vector<uint32_t> cuts{0};
    {
        long double total = 0, run = 0;
        for (uint32_t t : P.order) total += (long double)P.t_n[t] * P.t_nb[t] + P.t_n[t];
        // about 6e10 units run in twenty-five seconds; at least two launches,
        // so that every build goes through the same sliced path
        const int n_slices = (int)std::min<long double>(64, std::max<long double>(2, total / 6e10L + 1));
        for (uint32_t w = 0; w < P.order.size(); ++w) {
            const uint32_t t = P.order[w];
            run += (long double)P.t_n[t] * P.t_nb[t] + P.t_n[t];
            if (run * n_slices >= total * (long double)cuts.size() && cuts.size() < (size_t)n_slices) cuts.push_back(w + 1);
        }
        if (cuts.back() != P.order.size()) cuts.push_back((uint32_t)P.order.size());
    }
    auto t0 = std::chrono::steady_clock::now();
    flags = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        const uint32_t* order0 = a.order;
        for (size_t sl = 0; sl + 1 < cuts.size(); ++sl) {
            BuildArgs as = a;
            as.order = order0 + cuts[sl];
            as.n_work = cuts[sl + 1] - cuts[sl];
            if (hipMemset(d_q, 0, 4) != hipSuccess) return fail(SEISMIC_EHIP, "gpu build: memset failed");
            hipLaunchKernelGGL(seismic_dev::k_build_terms, dim3(grid), dim3(seismic_dev::kBT), 0, nullptr, as);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
                return fail(SEISMIC_EHIP, "gpu build: kernel failed");
            if (p->verbose && cuts.size() > 3)
                std::fprintf(stderr, "gpu build: lists %u..%u of %zu done (%.1f s)\n", cuts[sl], cuts[sl + 1],
                             P.order.size(),
                             std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        }
        (void)hipMemcpy(&flags, a.flags, 4, hipMemcpyDeviceToHost);
        if (flags != 4u || attempt == 1) break;
        // only the summary region was short: run again with its exact size
        unsigned long long need = 0;
        (void)hipMemcpy(&need, a.sum_bump, 8, hipMemcpyDeviceToHost);
        if (p->verbose) std::fprintf(stderr, "gpu build: %llu summary entries, rerunning with room for them\n", need);
        F.drop(a.sum_term);
        F.drop(a.sum_code);
        a.sum_cap = need;
        rc = dalloc(F.p, a.sum_term, need);
        if (!rc) rc = dalloc(F.p, a.sum_code, need);
        if (rc) return rc;
        ok = hipMemset(d_q, 0, 4) == hipSuccess && hipMemset(a.sum_bump, 0, 8) == hipSuccess &&
             hipMemset(a.flags, 0, 4) == hipSuccess && hipMemset(a.t_nblk, 0, (size_t)dim * 4) == hipSuccess;
        if (!ok) return fail(SEISMIC_EHIP, "gpu build: memset failed");
    }
    // the per-workgroup scratch is no longer needed
    for (void* x : {(void*)a.s_perm, (void*)a.s_assign, (void*)a.s_tcount, (void*)a.s_tstart, (void*)a.s_tfill,
                    (void*)a.s_touched, (void*)a.s_phi, (void*)a.s_ck, (void*)a.s_cv, (void*)a.s_sort})
        F.drop(x);
    return SEISMIC_OK;
}

// The per-block outputs in canonical order (terms ascending, each term's
// blocks in slot order) written into H's per-block arrays; src_at[j] =
// where canonical block j's summary sits in the kernel's bump region.
int canonical_blocks(const BuildArgs& a, const uint64_t* d_bsat, const Plan& P, uint32_t dim, HostIndex& H,
                     std::vector<uint64_t>& src_at, uint64_t& used) {
    const uint64_t total_b = P.total_b;
    std::vector<uint32_t> nblk(dim), b_len(total_b), b_cent(total_b), b_sum_len(total_b);
    std::vector<float> b_m(total_b), b_delta(total_b);
    std::vector<uint64_t> b_sum_at(total_b);
    used = 0;
    bool ok = hipMemcpy(nblk.data(), a.t_nblk, dim * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_len.data(), a.b_len, total_b * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_cent.data(), a.b_cent, total_b * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_sum_len.data(), a.b_sum_len, total_b * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_m.data(), a.b_m, total_b * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_delta.data(), a.b_delta, total_b * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b_sum_at.data(), d_bsat, total_b * 8, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&used, a.sum_bump, 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) return fail(SEISMIC_EHIP, "gpu build: download failed");
    H.list_off.assign(dim + 1, 0);
    for (uint32_t t = 0; t < dim; ++t) H.list_off[t + 1] = H.list_off[t] + nblk[t];
    const uint64_t nbt = H.list_off[dim];
    H.blk_post_off.assign(nbt + 1, 0);
    H.blk_sum_off.assign(nbt + 1, 0);
    H.blk_m.resize(nbt);
    H.blk_delta.resize(nbt);
    H.blk_centroid.resize(nbt);
    src_at.resize(nbt);
    for (uint32_t t = 0; t < dim; ++t)
        for (uint32_t j = 0; j < nblk[t]; ++j) {
            const uint64_t src = P.t_bcap[t] + j, dst = H.list_off[t] + j;
            H.blk_post_off[dst + 1] = H.blk_post_off[dst] + b_len[src];
            H.blk_sum_off[dst + 1] = H.blk_sum_off[dst] + b_sum_len[src];
            H.blk_m[dst] = b_m[src];
            H.blk_delta[dst] = b_delta[src];
            H.blk_centroid[dst] = b_cent[src];
            src_at[dst] = b_sum_at[src];
        }
    return SEISMIC_OK;
}

void set_params(HostIndex& H, const seismic_csr* docs, const seismic_build_params* p) {
    H.dim = docs->dim;
    H.n_docs = docs->n_rows;
    H.lambda = p->lambda;
    H.beta = p->beta;
    H.gamma = p->gamma;
    H.seed = p->seed;
    H.alpha = p->alpha;
}

int check_build_params(const seismic_build_params* p) {
    if (p->lambda < 1) return fail(SEISMIC_EINVAL, "build: lambda must be >= 1");
    if (p->beta < 1) return fail(SEISMIC_EINVAL, "build: beta must be >= 1");
    if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return fail(SEISMIC_EINVAL, "build: gamma must be in (0, 1]");
    if (!(p->alpha >= 0.0 && p->alpha <= 1.0)) return fail(SEISMIC_EINVAL, "build: alpha must be in [0, 1]");
    return SEISMIC_OK;
}

// A wave per canonical block copies its summary out of the bump region.
__global__ __launch_bounds__(256) void k_gather_sums(const uint64_t* src_at, const uint64_t* dst_off, uint64_t nbt,
                                                     const uint16_t* st, const uint8_t* sc, uint16_t* ot,
                                                     uint8_t* oc) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; j < nbt; j += waves) {
        const uint64_t at = src_at[j], to = dst_off[j], len = dst_off[j + 1] - to;
        for (uint64_t e = lane; e < len; e += kWave) {
            ot[to + e] = st[at + e];
            oc[to + e] = sc[at + e];
        }
    }
}

template <typename T>
int index_buffer(DeviceIndex* d, size_t n, size_t pad, const T*& out, T** mut = nullptr) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>((n + pad) * sizeof(T), 16);
    if (hipMalloc(&p, bytes) != hipSuccess)
        return fail(SEISMIC_ENOMEM, "device build: index allocation of %zu bytes failed", bytes);
    d->allocs.push_back(p);
    if (pad && hipMemset((uint8_t*)p + n * sizeof(T), 0, bytes - n * sizeof(T)) != hipSuccess)
        return fail(SEISMIC_EHIP, "device build: memset failed");
    out = (const T*)p;
    if (mut) *mut = (T*)p;
    return SEISMIC_OK;
}

template <typename T>
int index_upload(DeviceIndex* d, const std::vector<T>& v, const T*& out) {
    T* p = nullptr;
    int rc = index_buffer(d, v.size(), 0, out, &p);
    if (!rc && !v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(SEISMIC_EHIP, "device build: upload failed");
    return rc;
}

}  // namespace

extern "C" int seismic_build_index_gpu(const seismic_csr* docs, const seismic_build_params* p, int device,
                                       seismic_index** out) {
    using namespace seismic_dev;
    if (!out || !p || !docs) return fail(SEISMIC_EINVAL, "gpu build: null argument");
    *out = nullptr;
    int rc = check_build_params(p);
    if (!rc) rc = validate_csr_host(docs, 65536, "build: docs");
    if (rc) return rc;
    if (docs->n_rows >= 0xFFFFFFFFull) return fail(SEISMIC_EINVAL, "build: more than 2^32-1 documents");
    DeviceGuard g(device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "gpu build: cannot select device %d", device);
    auto t_start = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
    seismic_index* ix = new (std::nothrow) seismic_index();
    if (!ix) return fail(SEISMIC_ENOMEM, "gpu build: host allocation failed");
    HostIndex& H = ix->h;
    const uint32_t dim = docs->dim;
    const int nthreads = resolve_threads(p->n_threads);
    try {
        set_params(H, docs, p);
        H.row_ptr.assign(docs->row_ptr, docs->row_ptr + docs->n_rows + 1);
        H.words.assign(docs->words, docs->words + docs->nnz);
    } catch (const std::bad_alloc&) {
        delete ix;
        return fail(SEISMIC_ENOMEM, "gpu build: host allocation failed");
    }
    uint32_t row_max = 1;
    for (uint64_t d = 0; d < H.n_docs; ++d) row_max = std::max<uint32_t>(row_max, (uint32_t)(H.row_ptr[d + 1] - H.row_ptr[d]));
    Frees F;
    uint64_t* d_rp = nullptr;
    uint32_t* d_w = nullptr;
    rc = dupload(F.p, d_rp, H.row_ptr.data(), H.row_ptr.size());
    if (!rc) rc = dupload(F.p, d_w, H.words.data(), H.words.size());
    DevCsc csc;
    std::vector<uint64_t> off;
    if (!rc) rc = device_csc(d_rp, d_w, H.n_docs, dim, csc, &off);
    if (rc) { delete ix; return rc; }
    Plan P;
    plan_terms(off, dim, p, P);
    if (!plan_fits(P)) {
        csc.release();
        delete ix;
        return fail(SEISMIC_EINVAL, "gpu build: a list needs %u blocks or %u postings (the GPU build handles %u and %u); "
                    "build it with seismic_build_index", P.nb_max, P.n_max, kMaxNb, 1u << 24);
    }
    if (p->verbose) std::fprintf(stderr, "gpu build: column lists on the device (%.1f s)\n", elapsed());
    BuildArgs a;
    uint32_t flags = 0;
    uint64_t* d_bsat = nullptr;
    rc = run_terms(d_rp, d_w, dim, row_max, csc, P, p, device, F, a, flags, d_bsat);
    csc.release();
    if (rc) { delete ix; return rc; }
    if (flags) {
        delete ix;
        return fail(SEISMIC_EINVAL, "gpu build: a list exceeded the kernel's capacities (%u); build it with "
                    "seismic_build_index", flags);
    }
    if (p->verbose) std::fprintf(stderr, "gpu build: lists, blocks and summaries on the device (%.1f s)\n", elapsed());
    // assemble the host index in canonical order
    try {
        std::vector<uint64_t> src_at;
        uint64_t used = 0;
        rc = canonical_blocks(a, d_bsat, P, dim, H, src_at, used);
        if (rc) { delete ix; return rc; }
        H.postings.resize(P.total_n);
        bool ok = true;
        if (P.total_n) ok = hipMemcpy(H.postings.data(), a.postings, P.total_n * 4, hipMemcpyDeviceToHost) == hipSuccess;
        std::vector<uint16_t> st(used);
        std::vector<uint8_t> sc(used);
        if (ok && used)
            ok = hipMemcpy(st.data(), a.sum_term, used * 2, hipMemcpyDeviceToHost) == hipSuccess &&
                 hipMemcpy(sc.data(), a.sum_code, used, hipMemcpyDeviceToHost) == hipSuccess;
        if (!ok) { delete ix; return fail(SEISMIC_EHIP, "gpu build: download failed"); }
        const uint64_t nbt = H.list_off[dim];
        H.sum_term.resize(H.blk_sum_off[nbt]);
        H.sum_code.resize(H.blk_sum_off[nbt]);
        parallel_for((int64_t)nbt, nthreads, 4096, [&](int64_t j, int) {
            const uint64_t len = H.blk_sum_off[j + 1] - H.blk_sum_off[j], at = src_at[j], to = H.blk_sum_off[j];
            std::memcpy(H.sum_term.data() + to, st.data() + at, len * 2);
            std::memcpy(H.sum_code.data() + to, sc.data() + at, len);
        });
    } catch (const std::bad_alloc&) {
        delete ix;
        return fail(SEISMIC_ENOMEM, "gpu build: host allocation failed");
    }
    if (p->verbose) std::fprintf(stderr, "gpu build: done (%.1f s)\n", elapsed());
    *out = ix;
    return SEISMIC_OK;
}

extern "C" int seismic_build_index_device(const seismic_csr* docs, const seismic_build_params* p, int device,
                                          seismic_index** out) {
    using namespace seismic_dev;
    if (!out || !p || !docs) return fail(SEISMIC_EINVAL, "device build: null argument");
    *out = nullptr;
    int rc = check_build_params(p);
    if (rc) return rc;
    if (docs->n_rows >= 0xFFFFFFFFull) return fail(SEISMIC_EINVAL, "build: more than 2^32-1 documents");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(SEISMIC_EINVAL, "device build: device %d of %d", device, ndev);
    DeviceGuard g(device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "device build: cannot select device %d", device);
    auto t_start = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
    uint32_t row_max = 0;
    rc = validate_csr_device(docs, 65536, "device build: docs", &row_max);
    if (rc) return rc;
    const uint32_t dim = docs->dim;
    const uint64_t n_docs = docs->n_rows, nnz = docs->nnz;
    DevCsc csc;
    std::vector<uint64_t> off;
    rc = device_csc(docs->row_ptr, docs->words, n_docs, dim, csc, &off);
    if (rc) return rc;
    Plan P;
    plan_terms(off, dim, p, P);
    if (!plan_fits(P)) {
        csc.release();
        return fail(SEISMIC_EINVAL, "device build: a list needs %u blocks or %u postings (at most %u and %u)", P.nb_max,
                    P.n_max, kMaxNb, 1u << 24);
    }
    if (p->verbose) std::fprintf(stderr, "device build: column lists (%.1f s)\n", elapsed());
    Frees F;
    BuildArgs a;
    uint32_t flags = 0;
    uint64_t* d_bsat = nullptr;
    rc = run_terms(docs->row_ptr, docs->words, dim, row_max, csc, P, p, device, F, a, flags, d_bsat);
    csc.release();
    if (rc) return rc;
    if (flags) return fail(SEISMIC_EINVAL, "device build: a list exceeded the kernel's capacities (%u)", flags);
    F.drop(a.list_docs);
    if (p->verbose) std::fprintf(stderr, "device build: lists, blocks and summaries (%.1f s)\n", elapsed());
    seismic_index* ix = new (std::nothrow) seismic_index();
    if (!ix) return fail(SEISMIC_ENOMEM, "device build: host allocation failed");
    HostIndex& H = ix->h;
    std::vector<uint64_t> src_at;
    uint64_t used = 0;
    try {
        set_params(H, docs, p);
        rc = canonical_blocks(a, d_bsat, P, dim, H, src_at, used);
    } catch (const std::bad_alloc&) {
        rc = fail(SEISMIC_ENOMEM, "device build: host allocation failed");
    }
    if (rc) { delete ix; return rc; }
    const uint64_t nbt = H.list_off[dim], n_sums = H.blk_sum_off[nbt];
    uint32_t mb = H.max_blocks_per_list(), cap = 2;
    while (cap < mb) cap <<= 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ix; return fail(SEISMIC_EHIP, "device build: device query failed"); }
    DeviceIndex* d = new DeviceIndex();
    d->device = device;
    d->sort_cap = cap;
    d->smem_limit = prop.sharedMemPerBlock;
    ix->dev = d;
    ix->device_only = true;
    ix->dev_nnz = nnz;
    ix->dev_postings = P.total_n;
    ix->dev_sums = n_sums;
    seismic_dev::DevIdx& v = d->view;
    auto bail = [&](int code) {
        seismic_index_free(ix);
        return code;
    };
    // per-block arrays, then the summaries gathered into canonical order
    rc = index_upload(d, H.list_off, v.list_off);
    if (!rc) rc = index_upload(d, H.blk_post_off, v.blk_post_off);
    if (!rc) rc = index_upload(d, H.blk_sum_off, v.blk_sum_off);
    if (!rc) rc = index_upload(d, H.blk_m, v.blk_m);
    if (!rc) rc = index_upload(d, H.blk_delta, v.blk_delta);
    uint16_t* st = nullptr;
    uint8_t* sc = nullptr;
    if (!rc) rc = index_buffer(d, n_sums, 16, v.sum_term, &st);
    if (!rc) rc = index_buffer(d, n_sums, 16, v.sum_code, &sc);
    uint64_t* d_src = nullptr;
    if (!rc) rc = dupload(F.p, d_src, src_at.data(), src_at.size());
    if (rc) return bail(rc);
    if (nbt) {
        const uint64_t grid = std::min<uint64_t>(16384, (nbt + 3) / 4);
        hipLaunchKernelGGL(k_gather_sums, dim3((uint32_t)grid), dim3(256), 0, nullptr, d_src, v.blk_sum_off, nbt,
                           a.sum_term, a.sum_code, st, sc);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return bail(fail(SEISMIC_EHIP, "device build: summary gather failed"));
    }
    F.drop(a.sum_term);
    F.drop(a.sum_code);
    // the postings are already in canonical order
    F.take(a.postings);
    d->allocs.push_back(a.postings);
    v.postings = a.postings;
    // the forward index: a copy of the caller's rows (zero words after the end for vector loads)
    uint64_t* rp = nullptr;
    uint32_t* w = nullptr;
    rc = index_buffer(d, n_docs + 1, 0, v.row_ptr, &rp);
    if (!rc) rc = index_buffer(d, nnz, 8, v.words, &w);
    if (rc) return bail(rc);
    if (hipMemcpy(rp, docs->row_ptr, (n_docs + 1) * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
        (nnz && hipMemcpy(w, docs->words, nnz * 4, hipMemcpyDeviceToDevice) != hipSuccess))
        return bail(fail(SEISMIC_EHIP, "device build: forward index copy failed"));
    v.dim = dim;
    v.n_docs = (uint32_t)n_docs;
    rc = device_term_rank(d, H.list_off, dim);
    if (rc) return bail(rc);
    if (p->verbose) std::fprintf(stderr, "device build: done (%.1f s)\n", elapsed());
    *out = ix;
    return SEISMIC_OK;
}
