// Column lists of a device-resident collection, built on the device: the
// inverted index of Section 4.2 before any truncation (every posting of
// term t, document ascending), used by the index build (Algorithm
// "Indexing with Seismic") and by exact search.  Also the device-side
// validation of a document collection.
//
// A stable counting transpose in three kernels over chunks of kChunk
// documents:
//   count  a workgroup per chunk: per-term counts of the chunk (LDS
//          histograms over term ranges of kRange terms);
//   scan   a thread per term: each chunk's first position inside the term's
//          list (the counts of the earlier chunks), and the list length;
//   fill   a workgroup per chunk walks its documents in order; wave w owns
//          the terms t with t % 4 == w, so a term's postings are written by
//          one wave in document order, and a term never repeats inside a
//          row, so the wave's lanes never share a counter.
// Lists are therefore document-ascending without any sort.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "device_internal.h"

namespace seismic_dev {

namespace {

constexpr uint32_t kChunk = 16384;  // documents per chunk
constexpr uint32_t kRange = 16384;  // terms per LDS pass (64 KB of counters)
constexpr uint32_t kCT = 256;       // threads per workgroup
static_assert(kCT / kWave == 4, "fill assigns terms to 4 waves");

__global__ __launch_bounds__(kCT) void k_csc_count(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs,
                                                   uint32_t dim, uint32_t* cnt) {
    __shared__ uint32_t h[kRange];
    const uint32_t tid = threadIdx.x;
    const uint64_t c = blockIdx.x;
    const uint64_t d0 = c * kChunk, d1 = std::min<uint64_t>(n_docs, d0 + kChunk);
    const uint64_t w0 = row_ptr[d0], w1 = row_ptr[d1];
    for (uint32_t r0 = 0; r0 < dim; r0 += kRange) {
        const uint32_t r1 = std::min(dim, r0 + kRange);
        for (uint32_t i = tid; i < kRange; i += kCT) h[i] = 0;
        __syncthreads();
        for (uint64_t j = w0 + tid; j < w1; j += kCT) {
            const uint32_t t = words[j] & 0xFFFFu;
            if (t >= r0 && t < r1) atomicAdd(&h[t - r0], 1u);
        }
        __syncthreads();
        for (uint32_t t = r0 + tid; t < r1; t += kCT) cnt[c * dim + t] = h[t - r0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kCT) void k_csc_scan(uint32_t* cnt, uint64_t n_chunks, uint32_t dim, uint64_t* len) {
    const uint32_t t = blockIdx.x * kCT + threadIdx.x;
    if (t >= dim) return;
    uint64_t run = 0;
    for (uint64_t c = 0; c < n_chunks; ++c) {
        const uint32_t v = cnt[c * dim + t];
        cnt[c * dim + t] = (uint32_t)run;
        run += v;
    }
    len[t] = run;
}

__global__ __launch_bounds__(kCT) void k_csc_fill(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs,
                                                  uint32_t dim, const uint32_t* cnt, const uint64_t* off,
                                                  uint32_t* doc, uint16_t* val) {
    __shared__ uint32_t pos[kRange];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint64_t c = blockIdx.x;
    const uint64_t d0 = c * kChunk, d1 = std::min<uint64_t>(n_docs, d0 + kChunk);
    for (uint32_t r0 = 0; r0 < dim; r0 += kRange) {
        const uint32_t r1 = std::min(dim, r0 + kRange);
        for (uint32_t t = r0 + tid; t < r1; t += kCT) pos[t - r0] = cnt[c * dim + t];
        __syncthreads();
        for (uint64_t d = d0; d < d1; ++d) {
            const uint64_t a = row_ptr[d], b = row_ptr[d + 1];
            for (uint64_t j = a + lane; j < b; j += kWave) {
                const uint32_t w = words[j];
                const uint32_t t = w & 0xFFFFu;
                if (t < r0 || t >= r1 || (t & 3u) != wave) continue;
                const uint32_t p = pos[t - r0]++;
                const uint64_t at = off[t] + p;
                doc[at] = (uint32_t)d;
                val[at] = (uint16_t)(w >> 16);
            }
        }
        __syncthreads();
    }
}

// Per row: row_ptr monotone and inside [0, nnz], length <= max_len, terms
// < dim and strictly ascending, values positive finite fp16.  bad[0] = the
// first failing kind (atomicMax of a code), bad[1] = a failing row (low
// 32 bits), bad[2] = the longest row.
__global__ __launch_bounds__(kCT) void k_validate_rows(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_rows,
                                                       uint64_t nnz, uint32_t dim, uint32_t max_len, uint32_t* bad) {
    uint32_t longest = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kCT + threadIdx.x; i < n_rows; i += (uint64_t)gridDim.x * kCT) {
        const uint64_t a = row_ptr[i], b = row_ptr[i + 1];
        uint32_t kind = 0;
        if (b < a || b > nnz) kind = 1;
        else if (b - a > max_len) kind = 2;
        else {
            longest = std::max<uint32_t>(longest, (uint32_t)(b - a));
            uint32_t prev = 0;
            for (uint64_t j = a; j < b && !kind; ++j) {
                const uint32_t w = words[j], t = w & 0xFFFFu, h = w >> 16;
                if (t >= dim) kind = 3;
                else if (j > a && t <= prev) kind = 4;
                else if (h == 0 || h >= 0x7C00u) kind = 5;
                prev = t;
            }
        }
        if (kind) {
            atomicMax(&bad[0], kind);
            bad[1] = (uint32_t)i;
        }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) longest = std::max(longest, (uint32_t)__shfl_xor(longest, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&bad[2], longest);
}

}  // namespace

int validate_csr_device(const seismic_csr* m, uint32_t max_len, const char* what, uint32_t* row_max) {
    using seismic::fail;
    if (!m) return fail(SEISMIC_EINVAL, "%s: null matrix", what);
    if (!m->on_device) return fail(SEISMIC_EINVAL, "%s: device-resident rows required", what);
    if (m->dim < 1 || m->dim > 65536) return fail(SEISMIC_EINVAL, "%s: dim %u outside [1, 65536]", what, m->dim);
    if (!m->row_ptr) return fail(SEISMIC_EINVAL, "%s: null row_ptr", what);
    if (m->nnz && !m->words) return fail(SEISMIC_EINVAL, "%s: null words", what);
    uint64_t ends[2] = {1, 0};
    HIP_TRY(hipMemcpy(&ends[0], m->row_ptr, 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&ends[1], m->row_ptr + m->n_rows, 8, hipMemcpyDeviceToHost));
    if (ends[0] != 0 || ends[1] != m->nnz) return fail(SEISMIC_EINVAL, "%s: row_ptr must start at 0 and end at nnz", what);
    uint32_t* bad = nullptr;
    HIP_TRY(hipMalloc((void**)&bad, 16));
    uint32_t hb[4] = {0, 0, 0, 0};
    hipError_t e = hipMemset(bad, 0, 16);
    if (e == hipSuccess && m->n_rows) {
        const uint64_t grid = std::min<uint64_t>(8192, (m->n_rows + kCT - 1) / kCT);
        hipLaunchKernelGGL(k_validate_rows, dim3((uint32_t)grid), dim3(kCT), 0, nullptr, m->row_ptr, m->words, m->n_rows,
                           m->nnz, m->dim, max_len, bad);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e == hipSuccess) e = hipMemcpy(hb, bad, 16, hipMemcpyDeviceToHost);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(SEISMIC_EHIP, "%s: validation failed: %s", what, hipGetErrorString(e));
    if (hb[0]) {
        static const char* why[] = {"", "row_ptr not monotone", "row too long", "term id >= dim",
                                    "terms not strictly ascending", "value not finite and positive"};
        return fail(SEISMIC_EINVAL, "%s: row %u: %s", what, hb[1], why[std::min<uint32_t>(hb[0], 5)]);
    }
    if (row_max) *row_max = hb[2];
    return SEISMIC_OK;
}

int device_csc(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs, uint32_t dim, DevCsc& out,
               std::vector<uint64_t>* host_off) {
    using seismic::fail;
    out = DevCsc{};
    uint64_t nnz = 0;
    if (n_docs) HIP_TRY(hipMemcpy(&nnz, row_ptr + n_docs, 8, hipMemcpyDeviceToHost));
    const uint64_t n_chunks = std::max<uint64_t>(1, (n_docs + kChunk - 1) / kChunk);
    uint32_t* cnt = nullptr;
    uint64_t* len = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(cnt);
        (void)hipFree(len);
    };
    if (hipMalloc((void**)&cnt, std::max<size_t>(n_chunks * dim * 4, 16)) != hipSuccess ||
        hipMalloc((void**)&len, (size_t)dim * 8) != hipSuccess ||
        hipMalloc((void**)&out.off, ((size_t)dim + 1) * 8) != hipSuccess ||
        hipMalloc((void**)&out.doc, std::max<size_t>(nnz * 4, 16)) != hipSuccess ||
        hipMalloc((void**)&out.val, std::max<size_t>(nnz * 2, 16)) != hipSuccess) {
        cleanup();
        out.release();
        return fail(SEISMIC_ENOMEM, "column lists: device allocation of %llu postings failed", (unsigned long long)nnz);
    }
    std::vector<uint64_t> off(dim + 1, 0);
    hipError_t e = hipSuccess;
    if (n_docs) {
        hipLaunchKernelGGL(k_csc_count, dim3((uint32_t)n_chunks), dim3(kCT), 0, nullptr, row_ptr, words, n_docs, dim, cnt);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_csc_scan, dim3((dim + kCT - 1) / kCT), dim3(kCT), 0, nullptr, cnt, n_chunks, dim, len);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(off.data() + 1, len, (size_t)dim * 8, hipMemcpyDeviceToHost);
        for (uint32_t t = 0; t < dim; ++t) off[t + 1] += off[t];
        if (e == hipSuccess && off[dim] != nnz) {
            cleanup();
            out.release();
            return fail(SEISMIC_EINVAL, "column lists: counted %llu postings, row_ptr says %llu",
                        (unsigned long long)off[dim], (unsigned long long)nnz);
        }
    }
    if (e == hipSuccess) e = hipMemcpy(out.off, off.data(), off.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_docs) {
        hipLaunchKernelGGL(k_csc_fill, dim3((uint32_t)n_chunks), dim3(kCT), 0, nullptr, row_ptr, words, n_docs, dim, cnt,
                           out.off, out.doc, out.val);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    cleanup();
    if (e != hipSuccess) {
        out.release();
        return fail(SEISMIC_EHIP, "column lists: %s", hipGetErrorString(e));
    }
    if (host_off) host_off->swap(off);
    return SEISMIC_OK;
}

}  // namespace seismic_dev
