// Device-side runtime of libseismic: index upload, workspaces and the
// search / exact-search entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "device_internal.h"
#include "probe.h"

using namespace seismic;
using seismic_dev::DevIdx;

int device_index_layout(const DeviceIndex* d) { return !d ? 0 : !d->view.brow ? 1 : d->copy_all ? 2 : 3; }

void device_index_free(DeviceIndex* d) {
    if (!d) return;
    int prev = 0;
    bool switched = hipGetDevice(&prev) == hipSuccess && d->device >= 0 && hipSetDevice(d->device) == hipSuccess;
    for (void* p : d->allocs) (void)hipFree(p);
    (void)hipFree(d->csc_off);
    (void)hipFree(d->csc_doc);
    (void)hipFree(d->csc_val);
    (void)hipFree(d->xq_ptr);
    (void)hipFree(d->xq_words);
    if (d->xq_done) (void)hipEventDestroy(d->xq_done);
    (void)hipFree(d->knn);
    (void)hipFree(d->term_rank);
    if (switched) (void)hipSetDevice(prev);
    delete d;
}

int device_term_rank(DeviceIndex* d, const std::vector<uint32_t>& list_off, uint32_t dim) {
    std::vector<uint32_t> order(dim), rank(dim);
    for (uint32_t t = 0; t < dim; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return list_off[x + 1] - list_off[x] > list_off[y + 1] - list_off[y];
    });
    for (uint32_t i = 0; i < dim; ++i) rank[order[i]] = i;
    HIP_TRY(hipMalloc((void**)&d->term_rank, (size_t)dim * 4));
    HIP_TRY(hipMemcpy(d->term_rank, rank.data(), (size_t)dim * 4, hipMemcpyHostToDevice));
    return SEISMIC_OK;
}

namespace {

// pad: extra zeroed elements after the data (vector loads may overrun the
// last group of a section by up to pad elements)
template <typename T>
int upload_vec(DeviceIndex* d, const std::vector<T>& v, const T*& out, size_t pad = 0) {
    size_t bytes = std::max<size_t>((v.size() + pad) * sizeof(T), 16);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(SEISMIC_ENOMEM, "upload: hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    d->allocs.push_back(p);
    if (pad) {
        e = hipMemset((uint8_t*)p + v.size() * sizeof(T), 0, bytes - v.size() * sizeof(T));
        if (e != hipSuccess) return fail(SEISMIC_EHIP, "upload: hipMemset: %s", hipGetErrorString(e));
    }
    if (!v.empty()) {
        e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(SEISMIC_EHIP, "upload: hipMemcpy: %s", hipGetErrorString(e));
    }
    out = (const T*)p;
    return SEISMIC_OK;
}

}  // namespace

int grow(void** p, size_t& cap, size_t need, size_t elem) {
    if (need <= cap) return SEISMIC_OK;
    size_t n = std::max(need, cap * 2);
    (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(p, std::max<size_t>(n * elem, 16));
    if (e != hipSuccess) return fail(SEISMIC_ENOMEM, "staging: hipMalloc: %s", hipGetErrorString(e));
    cap = n;
    return SEISMIC_OK;
}

constexpr int kBuckets = 4;  // batch-size buckets of the launch configuration
constexpr uint32_t kMaxRefine = 256;  // refinement candidates per query (k * kappa), one workgroup pass

struct seismic_batch_graph {
    int device = -1;
    hipGraphExec_t exec = nullptr;
};

struct seismic_workspace {
    const seismic_index* index = nullptr;
    int device = -1;
    uint32_t max_queries = 0, max_k = 0;
    int n_cu = 0;
    seismic_launch_config cfg[kBuckets];
    uint32_t* queue = nullptr;  // device counter of the persistent search kernel
    double* probe_w = nullptr;  // sanitized learned-probe parameters of the current batch
    uint64_t* q_ptr = nullptr;  // staging for host-resident queries
    uint32_t* q_words = nullptr;
    size_t q_rows_cap = 0, q_words_cap = 0;
    seismic_dev::ListSched ls;  // list-major schedule buffers (allocated on first request)
    std::vector<void*> ls_allocs;
    seismic_dev::WideSched wd;  // wide schedule buffers (allocated on first request)
    std::vector<void*> wd_allocs;
};

namespace {

int bucket_of(uint64_t nq) { return nq <= 128 ? 0 : nq <= 256 ? 1 : nq <= 4096 ? 2 : 3; }

int check_config(const seismic_workspace* ws, const seismic_launch_config* c) {
    if (c->threads != 256 && c->threads != 512) return fail(SEISMIC_EINVAL, "config: threads must be 256 or 512");
    if (c->schedule > 2) return fail(SEISMIC_EINVAL, "config: schedule must be 0, 1 or 2");
    const uint32_t wmax = c->schedule == 2 ? seismic_dev::kWideMaxDepth : seismic_dev::kMaxW;
    if (c->window < 1 || c->window > wmax)
        return fail(SEISMIC_EINVAL, "config: window must be in [1, %u] for schedule %u", wmax, c->schedule);
    size_t smem = seismic_dev::search_smem_bytes(c->threads, ws->index->h.dim, ws->index->dev->sort_cap, ws->max_k);
    if (smem > ws->index->dev->smem_limit)
        return fail(SEISMIC_EINVAL, "config: %zu bytes of LDS needed, the device allows %zu", smem, ws->index->dev->smem_limit);
    return SEISMIC_OK;
}

int check_params(const seismic_index* index, const seismic_workspace* ws, const seismic_csr* queries,
                 const seismic_search_params* params) {
    if (!index->dev) return fail(SEISMIC_ESTATE, "search: index is not on a device");
    if (ws->index != index) return fail(SEISMIC_EINVAL, "search: workspace belongs to another index");
    if (params->k < 1 || params->k > ws->max_k) return fail(SEISMIC_EINVAL, "search: k = %u outside [1, %u]", params->k, ws->max_k);
    if (!(params->heap_factor > 0.0f)) return fail(SEISMIC_EINVAL, "search: heap_factor must be > 0");
    if (params->flags & ~SEISMIC_SEARCH_KNN) return fail(SEISMIC_EINVAL, "search: unknown flags");
    if (params->flags & SEISMIC_SEARCH_KNN) {
        if (!index->dev->knn) return fail(SEISMIC_ESTATE, "search: the index has no kappa-NN graph");
        if ((uint64_t)params->k * index->dev->kappa > kMaxRefine)
            return fail(SEISMIC_EINVAL, "search: refinement needs k * kappa <= %u (k %u, kappa %u)", kMaxRefine,
                        params->k, index->dev->kappa);
    }
    if (params->probe && !(params->probe_tau == params->probe_tau)) return fail(SEISMIC_EINVAL, "search: probe_tau is NaN");
    if (!(params->query_mass >= 0.0)) return fail(SEISMIC_EINVAL, "search: query_mass must be >= 0");
    if (queries->dim != index->h.dim) return fail(SEISMIC_EINVAL, "search: query dim %u != index dim %u", queries->dim, index->h.dim);
    if (queries->n_rows > ws->max_queries)
        return fail(SEISMIC_EINVAL, "search: %llu queries exceed the workspace (%u)", (unsigned long long)queries->n_rows, ws->max_queries);
    return SEISMIC_OK;
}

// Enqueue one search of device-resident rows with launch shape cfg.
// Buffers of the list-major schedule for the workspace's capacity.
int ensure_list_sched(seismic_workspace* ws) {
    if (ws->ls.cut) return SEISMIC_OK;
    const size_t nq = std::max<uint32_t>(ws->max_queries, 1), k = ws->max_k, R = seismic_dev::kMaxPositions;
    const uint32_t dim = ws->index->h.dim;
    seismic_dev::ListSched l;
    auto al = [&](auto*& p, size_t bytes) {
        void* x = nullptr;
        if (hipMalloc(&x, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        ws->ls_allocs.push_back(x);
        p = (std::remove_reference_t<decltype(p)>)x;
        return true;
    };
    bool ok = al(l.cut, nq * R * 2) && al(l.ncut, nq * 4) && al(l.hist, R * ((size_t)dim + 1) * 4) &&
              al(l.items, nq * R * 4) && al(l.key0, nq * 4) && al(l.seg, (R + 1) * 4) && al(l.queues, (R + 1) * 4) &&
              al(l.hs, nq * k * 4) && al(l.hid, nq * k * 4) && al(l.hn, nq * 4) && al(l.cnt, nq * 6 * 8);
    if (!ok) {
        for (void* x : ws->ls_allocs) (void)hipFree(x);
        ws->ls_allocs.clear();
        return fail(SEISMIC_ENOMEM, "workspace: list-major schedule buffers do not fit");
    }
    ws->ls = l;
    return SEISMIC_OK;
}

// Buffers of the wide schedule: up to kWideMaxBatch queries of the
// workspace, kWideMaxCut cut lists, kWideMaxDepth speculated blocks per list,
// top-k sets of min(max_k, kWideMaxK) entries.
int ensure_wide_sched(seismic_workspace* ws) {
    if (ws->wd.r) return SEISMIC_OK;
    seismic_dev::WideSched w;
    w.cap = std::max<uint32_t>(1, std::min(ws->max_queries, seismic_dev::kWideMaxBatch));
    w.sort_cap = ws->index->dev->sort_cap;
    w.k = std::min(ws->max_k, seismic_dev::kWideMaxK);
    const size_t lists = (size_t)w.cap * seismic_dev::kWideMaxCut, blocks = lists * seismic_dev::kWideMaxDepth;
    // evaluation items (chunks of kWideChunk documents) and their top-k
    // sets: up to four per speculated block within 256 MB of sets; a list
    // whose items do not fit speculates fewer blocks
    w.icap = (uint32_t)std::max<size_t>(blocks, std::min<size_t>(4 * blocks, (size_t(256) << 20) / (8 * w.k)));
    auto al = [&](auto*& p, size_t bytes) {
        void* x = nullptr;
        if (hipMalloc(&x, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        ws->wd_allocs.push_back(x);
        p = (std::remove_reference_t<decltype(p)>)x;
        return true;
    };
    bool ok = al(w.r, lists * w.sort_cap * 4) && al(w.ord, lists * w.sort_cap * 2) && al(w.nspec, lists * 4) &&
              al(w.items, (size_t)w.icap * 16) && al(w.cnt, 16) && al(w.first, blocks * 4) &&
              al(w.docs, blocks * 4) && al(w.nnz, blocks * 8) && al(w.ps, (size_t)w.icap * w.k * 4) &&
              al(w.pid, (size_t)w.icap * w.k * 4) && al(w.lb, (size_t)w.cap * 4) && al(w.fast, (size_t)w.cap * 4) &&
              al(w.cut, lists * 4);
    if (!ok) {
        for (void* x : ws->wd_allocs) (void)hipFree(x);
        ws->wd_allocs.clear();
        return fail(SEISMIC_ENOMEM, "workspace: wide schedule buffers do not fit");
    }
    ws->wd = w;
    return SEISMIC_OK;
}

// Does the wide schedule serve this batch (buffers present, sizes within them)?
bool wide_applies(const seismic_workspace* ws, uint64_t nq, const seismic_search_params* params, uint32_t nt) {
    const uint32_t dim = ws->index->h.dim, P = ws->index->dev->sort_cap;
    const size_t smem = seismic_dev::search_smem_bytes(nt, dim, P, params->k);
    const size_t smem_lists = seismic_dev::search_smem_bytes(seismic_dev::kWideListThreads, dim, P, params->k);
    return ws->wd.r && nq <= ws->wd.cap && params->query_cut >= 1 && params->query_cut <= seismic_dev::kWideMaxCut &&
           params->k <= ws->wd.k && smem + seismic_dev::kWideMetaBytes <= ws->index->dev->smem_limit &&
           smem_lists <= ws->index->dev->smem_limit;
}

int launch_batch(const seismic_index* index, seismic_workspace* ws, const uint64_t* q_ptr, const uint32_t* q_words,
                 uint64_t nq, uint64_t nnz, const seismic_search_params* params, uint32_t* out_ids, float* out_scores,
                 const seismic_stats* stats, const seismic_launch_config& cfg, hipStream_t st,
                 const uint32_t* nq_dev = nullptr) {
    seismic_dev::SearchArgs a{};
    a.nq_dev = nq_dev;
    a.ix = index->dev->view;
    a.q_ptr = q_ptr;
    a.q_words = q_words;
    a.q_nnz = nnz;
    a.k = params->k;
    a.cut = params->query_cut;
    a.qmass = params->query_mass;
    a.hf = params->heap_factor;
    a.sort_cap = index->dev->sort_cap;
    a.nq = (uint32_t)nq;
    a.window = cfg.window;
    a.queue = ws->queue;
    a.out_ids = out_ids;
    a.out_scores = out_scores;
    a.prefix = stats ? stats->prefix : nullptr;
    a.prefix_stride = stats ? stats->prefix_stride : 0;
    a.counters = stats ? stats->counters : nullptr;
    a.list_hmin = stats ? stats->list_hmin : nullptr;
    a.list_term = stats ? stats->list_term : nullptr;
    a.probe_w = nullptr;
    a.tau = params->probe_tau;
    if (params->probe) {
        HIP_TRY(seismic_dev::launch_probe_prep(params->probe, ws->probe_w, st));
        a.probe_w = ws->probe_w;
    }
    const uint32_t nt = cfg.threads;
    size_t smem = seismic_dev::search_smem_bytes(nt, index->h.dim, index->dev->sort_cap, params->k);
    int per_cu = seismic_dev::search_blocks_per_cu(nt, smem);
    if (per_cu < 1) return fail(SEISMIC_EHIP, "search: kernel does not fit on a CU (%zu bytes of LDS)", smem);
    if (cfg.blocks_per_cu > 0) per_cu = std::min<int>(per_cu, (int)cfg.blocks_per_cu);
    uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * (uint64_t)ws->n_cu, nq);
    if (cfg.schedule == 2 && wide_applies(ws, nq, params, nt)) {
        // a batch of at most kWideTinyBatch queries leaves most of the chip
        // idle: it speculates twice as deep (capped)
        a.depth_large = cfg.window;
        a.depth = std::min(2 * cfg.window, seismic_dev::kWideMaxDepth);
        const size_t smem_eval = seismic_dev::wide_eval_smem_bytes(index->h.dim, params->k);
        const int per_cu_eval = seismic_dev::wide_eval_blocks_per_cu(smem_eval);
        if (per_cu_eval < 1) return fail(SEISMIC_EHIP, "search: kernel does not fit on a CU (%zu bytes of LDS)", smem_eval);
        const size_t smem_lists = seismic_dev::search_smem_bytes(seismic_dev::kWideListThreads, index->h.dim,
                                                                 index->dev->sort_cap, params->k);
        HIP_TRY(seismic_dev::launch_search_wide(a, ws->wd, nt, (uint32_t)per_cu * (uint32_t)ws->n_cu, smem,
                                                2u * (uint32_t)ws->n_cu, smem_lists,
                                                (uint32_t)per_cu_eval * (uint32_t)ws->n_cu, smem_eval, st));
    } else if (cfg.schedule == 1 && ws->ls.cut && index->dev->term_rank && params->query_cut >= 1 &&
        params->query_cut <= seismic_dev::kMaxPositions) {
        seismic_dev::ListSched ls = ws->ls;
        ls.term_rank = index->dev->term_rank;
        HIP_TRY(seismic_dev::launch_search_positions(a, ls, nt, grid, smem, st));
    } else {
        HIP_TRY(seismic_dev::launch_search(a, nt, grid, smem, st));
    }
    if (params->flags & SEISMIC_SEARCH_KNN) {
        seismic_dev::RefineArgs r{};
        r.ix = a.ix;
        r.q_ptr = q_ptr;
        r.q_words = q_words;
        r.q_nnz = nnz;
        r.nq = a.nq;
        r.nq_dev = nq_dev;
        r.k = params->k;
        r.knn = index->dev->knn;
        r.kappa = index->dev->kappa;
        r.ids = out_ids;
        r.scores = out_scores;
        r.counters = a.counters;
        HIP_TRY(seismic_dev::launch_refine(r, st));
    }
    return SEISMIC_OK;
}

// Block-major copies of the rows of selected lists.  Selected list j holds
// the postings [gp[j], gp[j] + cb[j + 1] - cb[j]) and owns the copies
// [cb[j], cb[j + 1]), one per posting, in posting order: the rows of a block
// are one contiguous run.  Each row is padded with zero words to whole
// 16-byte groups.

// groups[j] = the 16-byte groups of list j's copies.  One workgroup per list.
__global__ __launch_bounds__(256) void k_copy_groups(const uint64_t* row_ptr, const uint32_t* postings,
                                                     const uint64_t* gp, const uint64_t* cb, uint64_t* groups) {
    __shared__ unsigned long long red[256 / seismic_dev::kWave];
    const uint32_t j = blockIdx.x;
    const uint64_t p0 = gp[j], n = cb[j + 1] - cb[j];
    unsigned long long s = 0;
    for (uint64_t i = threadIdx.x; i < n; i += 256) {
        const uint32_t d = postings[p0 + i];
        s += (row_ptr[d + 1] - row_ptr[d] + 3) / 4;
    }
    s = seismic_dev::wave_sum(s);
    if ((threadIdx.x & (seismic_dev::kWave - 1)) == 0) red[threadIdx.x / seismic_dev::kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / seismic_dev::kWave; ++w) t += red[w];
        groups[j] = t;
    }
}

// prow[c] = first group of copy c (list j's copies start at group
// gbase[j]), pnnz[c] = its nonzeros.  One workgroup per list, a scan over
// chunks of 256 copies with a running carry.
__global__ __launch_bounds__(256) void k_copy_offsets(const uint64_t* row_ptr, const uint32_t* postings,
                                                      const uint64_t* gp, const uint64_t* cb, const uint64_t* gbase,
                                                      uint64_t* prow, uint32_t* pnnz) {
    __shared__ uint32_t scratch[256 / seismic_dev::kWave];
    const uint32_t j = blockIdx.x;
    const uint64_t p0 = gp[j], c0 = cb[j], n = cb[j + 1] - c0;
    uint64_t carry = gbase[j];
    for (uint64_t base = 0; base < n; base += 256) {
        const uint64_t i = base + threadIdx.x;
        uint32_t len = 0;
        if (i < n) {
            const uint32_t d = postings[p0 + i];
            len = (uint32_t)(row_ptr[d + 1] - row_ptr[d]);
        }
        uint32_t tot;
        const uint32_t ex = seismic_dev::block_exscan<256>((len + 3) / 4, scratch, &tot);
        if (i < n) {
            prow[c0 + i] = carry + ex;
            pnnz[c0 + i] = len;
        }
        carry += tot;
    }
}

// The rows themselves: one wave per copy.
__global__ __launch_bounds__(256) void k_copy_rows(const uint64_t* row_ptr, const uint32_t* words,
                                                   const uint32_t* postings, const uint64_t* gp, const uint64_t* cb,
                                                   uint32_t n_lists, const uint64_t* prow, const uint32_t* pnnz,
                                                   uint32_t* brow) {
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / seismic_dev::kWave;
    const uint32_t lane = threadIdx.x & (seismic_dev::kWave - 1);
    const uint64_t n_waves = (uint64_t)gridDim.x * blockDim.x / seismic_dev::kWave, n = cb[n_lists];
    for (uint64_t c = wave; c < n; c += n_waves) {
        uint32_t lo = 0, hi = n_lists;  // the list of copy c: cb[lo] <= c < cb[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (cb[mid] <= c) lo = mid; else hi = mid;
        }
        const uint32_t d = postings[gp[lo] + (c - cb[lo])];
        const uint64_t rs = row_ptr[d], len = pnnz[c];
        const uint64_t dst = prow[c] * 4, m = (len + 3) / 4 * 4;
        for (uint64_t i = lane; i < m; i += seismic_dev::kWave) brow[dst + i] = i < len ? words[rs + i] : 0u;
    }
}

// Device buffers of one call, freed on every return unless released.
struct CallBuffers {
    std::vector<void*> p;
    ~CallBuffers() {
        if (p.empty()) return;
        (void)hipDeviceSynchronize();  // kernels of a failed call may still read them
        for (void* x : p) (void)hipFree(x);
    }
    int alloc(void** out, size_t bytes, const char* what) {
        *out = nullptr;
        hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 16));
        if (e != hipSuccess)
            return fail(SEISMIC_ENOMEM, "block-major copies: %s needs %zu bytes: %s", what, bytes, hipGetErrorString(e));
        p.push_back(*out);
        return SEISMIC_OK;
    }
    template <typename T>
    int put(T** out, const std::vector<T>& v, const char* what) {
        int rc = alloc((void**)out, v.size() * sizeof(T), what);
        if (!rc && !v.empty()) HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return rc;
    }
};

// Builds the copies of lists[0..n) (term ids, in priority order) for the
// longest prefix whose copies fit in max_bytes of device memory, counting
// the rows, 12 bytes of offsets per posting and the per-block map.
int build_copies(DeviceIndex* d, const HostIndex& h, const uint32_t* lists, uint32_t n, uint64_t max_bytes,
                 bool all, uint32_t* n_copied, uint64_t* bytes_used) {
    DevIdx& v = d->view;
    if (n_copied) *n_copied = 0;
    if (bytes_used) *bytes_used = 0;
    if (v.bcopy) return fail(SEISMIC_ESTATE, "block-major copies: the index already has them");
    if (n && !lists) return fail(SEISMIC_EINVAL, "block-major copies: null list array");
    std::vector<uint8_t> seen(h.dim, 0);
    for (uint32_t i = 0; i < n; ++i) {
        if (lists[i] >= h.dim) return fail(SEISMIC_EINVAL, "block-major copies: list %u >= dim %u", lists[i], h.dim);
        if (seen[lists[i]]++) return fail(SEISMIC_EINVAL, "block-major copies: list %u given twice", lists[i]);
    }
    // the selected lists that hold postings, with their postings and copies
    std::vector<uint32_t> term;
    std::vector<uint64_t> gp, cb(1, 0);
    auto empty = [&](uint32_t t) { return h.blk_post_off[h.list_off[t]] == h.blk_post_off[h.list_off[t + 1]]; };
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t t = lists[i];
        if (empty(t)) continue;
        const uint64_t p0 = h.blk_post_off[h.list_off[t]], np = h.blk_post_off[h.list_off[t + 1]] - p0;
        if (cb.back() + np >= seismic_dev::kNoCopy) {  // copy indexes are 32-bit
            if (all) return fail(SEISMIC_EINVAL, "block-major copies: more than 2^32 - 2 postings");
            break;
        }
        term.push_back(t);
        gp.push_back(p0);
        cb.push_back(cb.back() + np);
    }
    uint32_t J = (uint32_t)term.size();
    // entries of lists[] covered by the first J' selected lists: those
    // copied, and lists without postings among and right after them
    auto covered = [&](uint32_t Jc) {
        uint32_t i = 0, j = 0;
        while (i < n && (empty(lists[i]) || (j < Jc && lists[i] == term[j]))) {
            if (!empty(lists[i])) ++j;
            ++i;
        }
        return i;
    };
    if (J == 0) {
        if (n_copied) *n_copied = covered(0);
        return SEISMIC_OK;
    }
    CallBuffers tmp;
    uint64_t *d_gp = nullptr, *d_cb = nullptr, *d_groups = nullptr;
    int rc = tmp.put(&d_gp, gp, "list offsets");
    if (!rc) rc = tmp.put(&d_cb, cb, "list offsets");
    if (!rc) rc = tmp.alloc((void**)&d_groups, (size_t)J * 8, "list sizes");
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy_groups, dim3(J), dim3(256), 0, nullptr, v.row_ptr, v.postings, d_gp, d_cb, d_groups);
    HIP_TRY(hipGetLastError());
    std::vector<uint64_t> groups(J);
    HIP_TRY(hipMemcpy(groups.data(), d_groups, (size_t)J * 8, hipMemcpyDeviceToHost));
    // the longest prefix that fits
    const uint64_t nb = h.list_off[h.dim];
    const uint64_t fixed = nb * 4 + 32;  // the block map and the rows' padding
    std::vector<uint64_t> gbase(J + 1, 0);
    uint32_t keep = 0;
    for (uint32_t j = 0; j < J; ++j) {
        gbase[j + 1] = gbase[j] + groups[j];
        const uint64_t need = fixed + gbase[j + 1] * 16 + cb[j + 1] * 12;
        if (!all && need > max_bytes) break;
        keep = j + 1;
    }
    if (keep == 0) {
        if (n_copied) *n_copied = covered(0);
        return SEISMIC_OK;
    }
    J = keep;
    const uint64_t nc = cb[J], ng = gbase[J];
    uint64_t *d_gbase = nullptr, *prow = nullptr;
    uint32_t *pnnz = nullptr, *brow = nullptr, *bcopy = nullptr;
    gbase.resize(J);
    rc = tmp.put(&d_gbase, gbase, "list offsets");
    if (!rc) rc = tmp.alloc((void**)&prow, nc * 8, "row offsets");
    if (!rc) rc = tmp.alloc((void**)&pnnz, nc * 4, "row lengths");
    // +2 groups: vector loads past the last row stay inside
    if (!rc) rc = tmp.alloc((void**)&brow, (ng + 2) * 16, "rows");
    if (!rc) rc = tmp.alloc((void**)&bcopy, nb * 4, "block map");
    if (rc) return rc;
    HIP_TRY(hipMemset((uint8_t*)brow + ng * 16, 0, 32));
    hipLaunchKernelGGL(k_copy_offsets, dim3(J), dim3(256), 0, nullptr, v.row_ptr, v.postings, d_gp, d_cb, d_gbase,
                       prow, pnnz);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_copy_rows, dim3(8192), dim3(256), 0, nullptr, v.row_ptr, v.words, v.postings, d_gp, d_cb, J,
                       prow, pnnz, brow);
    HIP_TRY(hipGetLastError());
    std::vector<uint32_t> map(nb, seismic_dev::kNoCopy);
    for (uint32_t j = 0; j < J; ++j)
        for (uint32_t b = h.list_off[term[j]]; b < h.list_off[term[j] + 1]; ++b)
            map[b] = (uint32_t)(cb[j] + (h.blk_post_off[b] - gp[j]));
    HIP_TRY(hipMemcpy(bcopy, map.data(), nb * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    // the copies now belong to the index
    for (void* x : {(void*)prow, (void*)pnnz, (void*)brow, (void*)bcopy}) {
        tmp.p.erase(std::find(tmp.p.begin(), tmp.p.end(), x));
        d->allocs.push_back(x);
    }
    v.prow = prow;
    v.pnnz = pnnz;
    v.brow = brow;
    v.bcopy = bcopy;
    std::vector<uint8_t> done(h.dim, 0);
    for (uint32_t j = 0; j < J; ++j) done[term[j]] = 1;
    d->copy_all = true;
    for (uint32_t t = 0; t < h.dim; ++t) d->copy_all = d->copy_all && (done[t] || empty(t));
    if (n_copied) *n_copied = covered(J);
    if (bytes_used) *bytes_used = fixed + ng * 16 + nc * 12;
    return SEISMIC_OK;
}

}  // namespace

namespace seismic {

int download_host_index(const seismic_index* ix, HostIndex& out) {
    const HostIndex& h = ix->h;
    const DeviceIndex* d = ix->dev;
    if (!d) return fail(SEISMIC_ESTATE, "download: index is not on a device");
    DeviceGuard g(d->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "download: cannot select device %d", d->device);
    out = HostIndex();
    out.dim = h.dim;
    out.n_docs = h.n_docs;
    out.lambda = h.lambda;
    out.beta = h.beta;
    out.gamma = h.gamma;
    out.seed = h.seed;
    out.alpha = h.alpha;
    out.list_off = h.list_off;
    out.blk_post_off = h.blk_post_off;
    out.blk_sum_off = h.blk_sum_off;
    out.blk_m = h.blk_m;
    out.blk_delta = h.blk_delta;
    out.blk_centroid = h.blk_centroid;
    out.row_ptr.resize(h.n_docs + 1);
    out.words.resize(ix->dev_nnz);
    out.postings.resize(ix->dev_postings);
    out.sum_term.resize(ix->dev_sums);
    out.sum_code.resize(ix->dev_sums);
    const seismic_dev::DevIdx& v = d->view;
    HIP_TRY(hipMemcpy(out.row_ptr.data(), v.row_ptr, out.row_ptr.size() * 8, hipMemcpyDeviceToHost));
    if (!out.words.empty()) HIP_TRY(hipMemcpy(out.words.data(), v.words, out.words.size() * 4, hipMemcpyDeviceToHost));
    if (!out.postings.empty())
        HIP_TRY(hipMemcpy(out.postings.data(), v.postings, out.postings.size() * 4, hipMemcpyDeviceToHost));
    if (!out.sum_term.empty()) {
        HIP_TRY(hipMemcpy(out.sum_term.data(), v.sum_term, out.sum_term.size() * 2, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(out.sum_code.data(), v.sum_code, out.sum_code.size(), hipMemcpyDeviceToHost));
    }
    return SEISMIC_OK;
}

int full_host_index(const seismic_index* ix, HostIndex& tmp, const HostIndex** out) {
    if (!ix->device_only) {
        *out = &ix->h;
        return SEISMIC_OK;
    }
    int rc;
    try {
        rc = download_host_index(ix, tmp);
    } catch (const std::bad_alloc&) {
        rc = fail(SEISMIC_ENOMEM, "download: host allocation failed");
    }
    if (!rc) *out = &tmp;
    return rc;
}

}  // namespace seismic

extern "C" {

int seismic_index_upload(seismic_index* index, int device, uint32_t flags) {
    if (!index) return fail(SEISMIC_EINVAL, "upload: null index");
    if (flags & ~SEISMIC_UPLOAD_BLOCK_ROWS) return fail(SEISMIC_EINVAL, "upload: unknown flags");
    std::lock_guard<std::mutex> lk(index->mu);
    if (index->dev) return fail(SEISMIC_ESTATE, "upload: index already on device %d", index->dev->device);
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(SEISMIC_EINVAL, "upload: device %d of %d", device, ndev);
    const HostIndex& h = index->h;
    uint32_t mb = h.max_blocks_per_list();
    uint32_t cap = 2;
    while (cap < mb) cap <<= 1;
    if (cap > seismic_dev::kMaxSortCap)
        return fail(SEISMIC_EINVAL, "upload: a list has %u blocks; at most %u are supported", mb, seismic_dev::kMaxSortCap);
    DeviceGuard g(device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "upload: cannot select device %d", device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    DeviceIndex* d = new DeviceIndex();
    d->device = device;
    d->sort_cap = cap;
    d->smem_limit = prop.sharedMemPerBlock;
    DevIdx& v = d->view;
    int rc = 0;
    if (!rc) rc = upload_vec(d, h.row_ptr, v.row_ptr);
    if (!rc) rc = upload_vec(d, h.words, v.words, 8);
    if (!rc) rc = upload_vec(d, h.list_off, v.list_off);
    if (!rc) rc = upload_vec(d, h.blk_post_off, v.blk_post_off);
    if (!rc) rc = upload_vec(d, h.blk_sum_off, v.blk_sum_off);
    if (!rc) rc = upload_vec(d, h.blk_m, v.blk_m);
    if (!rc) rc = upload_vec(d, h.blk_delta, v.blk_delta);
    if (!rc) rc = upload_vec(d, h.postings, v.postings);
    if (!rc) rc = upload_vec(d, h.sum_term, v.sum_term, 16);
    if (!rc) rc = upload_vec(d, h.sum_code, v.sum_code, 16);
    if (!rc && (flags & SEISMIC_UPLOAD_BLOCK_ROWS)) {
        std::vector<uint32_t> all(h.dim);
        for (uint32_t t = 0; t < h.dim; ++t) all[t] = t;
        rc = build_copies(d, h, all.data(), h.dim, 0, true, nullptr, nullptr);
    }
    if (!rc) rc = device_term_rank(d, h.list_off, h.dim);
    if (rc) { device_index_free(d); return rc; }
    v.dim = h.dim;
    v.n_docs = (uint32_t)h.n_docs;
    index->dev = d;
    return SEISMIC_OK;
}

int seismic_index_copy_lists(seismic_index* index, const uint32_t* lists, uint32_t n_lists, uint64_t max_bytes,
                             uint32_t* n_copied, uint64_t* bytes) {
    if (!index) return fail(SEISMIC_EINVAL, "copy lists: null index");
    std::lock_guard<std::mutex> lk(index->mu);
    if (!index->dev) return fail(SEISMIC_ESTATE, "copy lists: index is not on a device");
    DeviceGuard g(index->dev->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "copy lists: cannot select device %d", index->dev->device);
    return build_copies(index->dev, index->h, lists, n_lists, max_bytes, false, n_copied, bytes);
}

int seismic_index_release_exact(seismic_index* index) {
    if (!index) return fail(SEISMIC_EINVAL, "release exact: null index");
    std::lock_guard<std::mutex> lk(index->mu);
    DeviceIndex* d = index->dev;
    if (!d || !d->csc_off) return SEISMIC_OK;
    DeviceGuard g(d->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "release exact: cannot select device %d", d->device);
    HIP_TRY(hipDeviceSynchronize());  // exact searches in flight still read them
    (void)hipFree(d->csc_off);
    (void)hipFree(d->csc_doc);
    (void)hipFree(d->csc_val);
    d->csc_off = nullptr;
    d->csc_doc = nullptr;
    d->csc_val = nullptr;
    return SEISMIC_OK;
}

int seismic_workspace_create(const seismic_index* index, uint32_t max_queries, uint32_t max_k, seismic_workspace** out) {
    if (!index || !out) return fail(SEISMIC_EINVAL, "workspace: null argument");
    *out = nullptr;
    if (!index->dev) return fail(SEISMIC_ESTATE, "workspace: index is not on a device");
    if (max_k < 1 || max_k > SEISMIC_MAX_K) return fail(SEISMIC_EINVAL, "workspace: max_k must be in [1, %d]", SEISMIC_MAX_K);
    seismic_workspace* ws = new (std::nothrow) seismic_workspace();
    if (!ws) return fail(SEISMIC_ENOMEM, "workspace: host allocation failed");
    ws->index = index;
    ws->device = index->dev->device;
    ws->max_queries = max_queries;
    ws->max_k = max_k;
    // default shapes: a batch of up to 128 queries runs the wide schedule
    // (512-thread list pass and traversal, 32 speculated blocks per list: at
    // 8.8M, 0.25 ms for one query, 0.85 ms for 32 and 1.66 ms for 96,
    // against 1.6, 2.0 and 2.1 ms query-major; even at 128), up to 256
    // queries one query per CU with 512-thread workgroups, larger batches
    // 256-thread workgroups, three per CU; the autotuner can replace any of
    // them
    ws->cfg[0] = seismic_launch_config{512u, 0, 32u, 2u};
    ws->cfg[1] = seismic_launch_config{512u, 0, 16u, 0};
    for (int b = 2; b < kBuckets; ++b) ws->cfg[b] = seismic_launch_config{256u, 0, 8u, 0};
    int rc = check_config(ws, &ws->cfg[2]);
    if (rc) { delete ws; return rc; }
    if (check_config(ws, &ws->cfg[1]) != SEISMIC_OK) ws->cfg[1] = ws->cfg[2];  // 512 threads do not fit
    if (check_config(ws, &ws->cfg[0]) != SEISMIC_OK) {
        ws->cfg[0].threads = 256;
        if (check_config(ws, &ws->cfg[0]) != SEISMIC_OK) ws->cfg[0] = ws->cfg[2];
    }
    clear_error();
    DeviceGuard g(ws->device);
    hipDeviceProp_t prop;
    if (!g.ok() || hipGetDeviceProperties(&prop, ws->device) != hipSuccess) {
        delete ws;
        return fail(SEISMIC_EHIP, "workspace: cannot query device %d", index->dev->device);
    }
    ws->n_cu = prop.multiProcessorCount;
    if (hipMalloc((void**)&ws->queue, 256) != hipSuccess ||
        hipMalloc((void**)&ws->probe_w, seismic_dev::kProbeWords * sizeof(double)) != hipSuccess) {
        (void)hipFree(ws->queue);
        delete ws;
        return fail(SEISMIC_ENOMEM, "workspace: device allocation failed");
    }
    *out = ws;
    return SEISMIC_OK;
}

void seismic_workspace_free(seismic_workspace* ws) {
    if (!ws) return;
    DeviceGuard g(ws->device);
    (void)hipFree(ws->queue);
    (void)hipFree(ws->probe_w);
    (void)hipFree(ws->q_ptr);
    (void)hipFree(ws->q_words);
    for (void* x : ws->ls_allocs) (void)hipFree(x);
    for (void* x : ws->wd_allocs) (void)hipFree(x);
    delete ws;
}

int seismic_workspace_set_config(seismic_workspace* ws, const seismic_launch_config* cfg) {
    if (!ws || !cfg) return fail(SEISMIC_EINVAL, "config: null argument");
    int rc = check_config(ws, cfg);
    if (!rc && cfg->schedule >= 1) {
        DeviceGuard g(ws->device);
        rc = !g.ok() ? fail(SEISMIC_EHIP, "config: cannot select device")
                     : cfg->schedule == 1 ? ensure_list_sched(ws) : ensure_wide_sched(ws);
    }
    if (rc) return rc;
    for (auto& c : ws->cfg) c = *cfg;
    return SEISMIC_OK;
}

int seismic_workspace_get_config(const seismic_workspace* ws, uint32_t n_queries, seismic_launch_config* cfg) {
    if (!ws || !cfg) return fail(SEISMIC_EINVAL, "config: null argument");
    *cfg = ws->cfg[bucket_of(n_queries)];
    return SEISMIC_OK;
}

int seismic_workspace_resident_per_cu(const seismic_workspace* ws, uint32_t n_queries, uint32_t k, uint32_t* per_cu) {
    if (!ws || !per_cu) return fail(SEISMIC_EINVAL, "resident: null argument");
    if (k < 1 || k > ws->max_k) return fail(SEISMIC_EINVAL, "resident: k = %u outside [1, %u]", k, ws->max_k);
    const seismic_launch_config& c = ws->cfg[bucket_of(n_queries)];
    DeviceGuard g(ws->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "resident: cannot select device");
    // the occupancy query the search sizes its persistent grid by, for this
    // shape's threads and this k's LDS (with the wide schedule it sizes the
    // traversal's grid)
    const size_t smem = seismic_dev::search_smem_bytes(c.threads, ws->index->h.dim, ws->index->dev->sort_cap, k);
    int n = seismic_dev::search_blocks_per_cu(c.threads, smem);
    if (c.blocks_per_cu > 0) n = std::min<int>(n, (int)c.blocks_per_cu);
    *per_cu = (uint32_t)std::max(n, 0);
    return SEISMIC_OK;
}

int seismic_search_batch(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                         const seismic_search_params* params, uint32_t* out_ids, float* out_scores,
                         const seismic_stats* stats, void* stream) {
    if (!index || !ws || !queries || !params || !out_ids || !out_scores)
        return fail(SEISMIC_EINVAL, "search: null argument");
    int rc = check_params(index, ws, queries, params);
    if (rc) return rc;
    if (stats && stats->prefix && stats->prefix_stride < 1) return fail(SEISMIC_EINVAL, "search: prefix_stride must be >= 1");
    DeviceGuard g(ws->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "search: cannot select device");
    hipStream_t st = (hipStream_t)stream;
    const uint64_t* q_ptr = queries->row_ptr;
    const uint32_t* q_words = queries->words;
    if (!queries->on_device) {
        rc = validate_csr_host(queries, SEISMIC_MAX_QUERY_NNZ, "search: queries");
        if (rc) return rc;
        rc = grow((void**)&ws->q_ptr, ws->q_rows_cap, queries->n_rows + 1, sizeof(uint64_t));
        if (!rc) rc = grow((void**)&ws->q_words, ws->q_words_cap, std::max<uint64_t>(queries->nnz, 1), sizeof(uint32_t));
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(ws->q_ptr, queries->row_ptr, (queries->n_rows + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        if (queries->nnz)
            HIP_TRY(hipMemcpyAsync(ws->q_words, queries->words, queries->nnz * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        q_ptr = ws->q_ptr;
        q_words = ws->q_words;
    }
    const seismic_launch_config& cfg = ws->cfg[bucket_of(queries->n_rows)];
    if (cfg.schedule == 2 && !ws->wd.r) {
        // allocate the wide schedule's buffers unless the stream is being
        // captured (the batch then runs query-major)
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) (void)ensure_wide_sched(ws);
        clear_error();
    }
    return launch_batch(index, ws, q_ptr, q_words, queries->n_rows, queries->nnz, params, out_ids, out_scores, stats,
                        cfg, st);
}

int seismic_autotune(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                     const seismic_search_params* params, uint32_t* out_ids, float* out_scores, uint32_t reps,
                     seismic_tune_result* results, uint32_t max_results, uint32_t* n_results, void* stream) {
    if (!index || !ws || !queries || !params || !out_ids || !out_scores)
        return fail(SEISMIC_EINVAL, "autotune: null argument");
    if (!queries->on_device) return fail(SEISMIC_EINVAL, "autotune: queries must be device resident");
    int rc = check_params(index, ws, queries, params);
    if (rc) return rc;
    if (n_results) *n_results = 0;
    if (queries->n_rows == 0) return SEISMIC_OK;
    if (reps < 1) reps = 1;
    DeviceGuard g(ws->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "autotune: cannot select device");
    hipStream_t st = (hipStream_t)stream;
    const size_t n_out = (size_t)queries->n_rows * params->k;
    std::vector<uint32_t> ref_ids(n_out), ids(n_out);
    std::vector<float> ref_sc(n_out), sc(n_out);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = INFINITY;
    seismic_launch_config best_cfg = ws->cfg[bucket_of(queries->n_rows)];
    uint32_t count = 0;
    bool have_ref = false;
    int err = SEISMIC_OK;
    // the list-major schedule is tried when it applies and its buffers fit
    const bool lists = params->query_cut >= 1 && params->query_cut <= seismic_dev::kMaxPositions &&
                       index->dev->term_rank && ensure_list_sched(ws) == SEISMIC_OK;
    // the wide schedule for small batches (speculation depths 8..64, full grid)
    const bool wide = queries->n_rows <= seismic_dev::kWideMaxBatch && ensure_wide_sched(ws) == SEISMIC_OK &&
                      wide_applies(ws, queries->n_rows, params, 256);
    clear_error();
    for (uint32_t sched = 0; sched <= 2 && !err; ++sched)
    for (uint32_t nt : {256u, 512u}) {
        if ((sched == 1 && !lists) || (sched == 2 && !wide)) break;
        size_t smem = seismic_dev::search_smem_bytes(nt, index->h.dim, index->dev->sort_cap, params->k);
        if (smem > index->dev->smem_limit) continue;
        if (sched == 2 && !wide_applies(ws, queries->n_rows, params, nt)) continue;
        const int max_pc = seismic_dev::search_blocks_per_cu(nt, smem);
        for (int pc = sched == 2 ? max_pc : 1; pc <= max_pc && !err; ++pc) {
            static const uint32_t kWindows[5] = {1, 2, 4, 8, 16}, kDepths[4] = {8, 16, 32, 64};
            const uint32_t* wl = sched == 2 ? kDepths : kWindows;
            const int n_wl = sched == 2 ? 4 : 5;
            for (int wi = 0; wi < n_wl; ++wi) {
                const uint32_t w = wl[wi];
                seismic_launch_config c{nt, (uint32_t)pc, w, sched};
                // warm-up run, then compare its results with the first shape's
                err = launch_batch(index, ws, queries->row_ptr, queries->words, queries->n_rows, queries->nnz, params,
                                   out_ids, out_scores, nullptr, c, st);
                if (err) break;
                if (hipMemcpyAsync(have_ref ? ids.data() : ref_ids.data(), out_ids, n_out * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipMemcpyAsync(have_ref ? sc.data() : ref_sc.data(), out_scores, n_out * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    err = fail(SEISMIC_EHIP, "autotune: copy of results failed");
                    break;
                }
                if (have_ref && (std::memcmp(ids.data(), ref_ids.data(), n_out * 4) != 0 ||
                                 std::memcmp(sc.data(), ref_sc.data(), n_out * 4) != 0)) {
                    err = fail(SEISMIC_ESTATE, "autotune: results differ between launch shapes (threads %u, per CU %d, window %u, schedule %u)", nt, pc, w, sched);
                    break;
                }
                have_ref = true;
                if (hipEventRecord(e0, st) != hipSuccess) { err = fail(SEISMIC_EHIP, "autotune: event record failed"); break; }
                for (uint32_t r = 0; r < reps && !err; ++r)
                    err = launch_batch(index, ws, queries->row_ptr, queries->words, queries->n_rows, queries->nnz, params,
                                       out_ids, out_scores, nullptr, c, st);
                if (err) break;
                float ms = 0.0f;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    err = fail(SEISMIC_EHIP, "autotune: event timing failed");
                    break;
                }
                ms /= (float)reps;
                if (results && count < max_results) results[count] = seismic_tune_result{c, ms, 0};
                ++count;
                if (ms < best) { best = ms; best_cfg = c; }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err) return err;
    ws->cfg[bucket_of(queries->n_rows)] = best_cfg;
    if (n_results) *n_results = std::min(count, max_results);
    return SEISMIC_OK;
}

int seismic_graph_create(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                         const uint32_t* n_queries_dev, const seismic_search_params* params, uint32_t* out_ids,
                         float* out_scores, const seismic_stats* stats, seismic_batch_graph** out) {
    if (!index || !ws || !queries || !n_queries_dev || !params || !out_ids || !out_scores || !out)
        return fail(SEISMIC_EINVAL, "graph: null argument");
    *out = nullptr;
    if (!queries->on_device) return fail(SEISMIC_EINVAL, "graph: queries must be device resident");
    int rc = check_params(index, ws, queries, params);
    if (rc) return rc;
    if (queries->n_rows == 0) return fail(SEISMIC_EINVAL, "graph: capacity of 0 queries");
    if (stats && stats->prefix && stats->prefix_stride < 1) return fail(SEISMIC_EINVAL, "graph: prefix_stride must be >= 1");
    DeviceGuard g(ws->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "graph: cannot select device");
    seismic_batch_graph* gr = new (std::nothrow) seismic_batch_graph();
    if (!gr) return fail(SEISMIC_ENOMEM, "graph: host allocation failed");
    gr->device = ws->device;
    if (ws->cfg[bucket_of(queries->n_rows)].schedule == 2) (void)ensure_wide_sched(ws);  // before capture
    clear_error();
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        delete gr;
        return fail(SEISMIC_EHIP, "graph: begin capture: %s", hipGetErrorString(e));
    }
    rc = launch_batch(index, ws, queries->row_ptr, queries->words, queries->n_rows, queries->nnz, params, out_ids,
                      out_scores, stats, ws->cfg[bucket_of(queries->n_rows)], cs, n_queries_dev);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete gr;
        return rc ? rc : fail(SEISMIC_EHIP, "graph: end capture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        delete gr;
        return fail(SEISMIC_EHIP, "graph: instantiate: %s", hipGetErrorString(e));
    }
    *out = gr;
    return SEISMIC_OK;
}

int seismic_graph_launch(seismic_batch_graph* graph, void* stream) {
    if (!graph) return fail(SEISMIC_EINVAL, "graph: null graph");
    DeviceGuard g(graph->device);
    HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return SEISMIC_OK;
}

void seismic_graph_free(seismic_batch_graph* graph) {
    if (!graph) return;
    DeviceGuard g(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    delete graph;
}

int seismic_index_set_knn(seismic_index* index, uint32_t kappa, const uint32_t* table, uint32_t on_device) {
    if (!index || !table) return fail(SEISMIC_EINVAL, "set_knn: null argument");
    if (!index->dev) return fail(SEISMIC_ESTATE, "set_knn: index is not on a device");
    if (kappa < 1 || kappa > kMaxRefine) return fail(SEISMIC_EINVAL, "set_knn: kappa must be in [1, %u]", kMaxRefine);
    DeviceIndex* d = index->dev;
    DeviceGuard g(d->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "set_knn: cannot select device");
    std::lock_guard<std::mutex> lk(index->mu);
    const size_t bytes = std::max<size_t>((size_t)index->h.n_docs * kappa * 4, 16);
    uint32_t* t = nullptr;
    if (hipMalloc((void**)&t, bytes) != hipSuccess) return fail(SEISMIC_ENOMEM, "set_knn: %zu bytes of device memory", bytes);
    hipError_t e = hipMemcpy(t, table, (size_t)index->h.n_docs * kappa * 4,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t);
        return fail(SEISMIC_EHIP, "set_knn: copy failed: %s", hipGetErrorString(e));
    }
    (void)hipFree(d->knn);
    d->knn = t;
    d->kappa = kappa;
    return SEISMIC_OK;
}

int seismic_index_get_knn(const seismic_index* index, uint32_t* out_host, uint32_t* kappa) {
    if (!index || !kappa) return fail(SEISMIC_EINVAL, "get_knn: null argument");
    *kappa = 0;
    if (!index->dev || !index->dev->knn) return SEISMIC_OK;
    *kappa = index->dev->kappa;
    if (!out_host) return SEISMIC_OK;
    DeviceGuard g(index->dev->device);
    HIP_TRY(hipMemcpy(out_host, index->dev->knn, (size_t)index->h.n_docs * index->dev->kappa * 4, hipMemcpyDeviceToHost));
    return SEISMIC_OK;
}

// Row u of the graph from the search of document u: its first kappa
// results other than u (0xFFFFFFFF padding kept).
__global__ void k_knn_finalize(const uint32_t* __restrict__ ids, uint32_t n, uint32_t first, uint32_t kappa,
                               uint32_t* __restrict__ table) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t u = first + i;
    const uint32_t* row = ids + (size_t)i * (kappa + 1);
    uint32_t* out = table + (size_t)u * kappa;
    uint32_t w = 0;
    for (uint32_t j = 0; j <= kappa && w < kappa; ++j)
        if (row[j] != u && row[j] != 0xFFFFFFFFu) out[w++] = row[j];
    for (; w < kappa; ++w) out[w] = 0xFFFFFFFFu;
}

int seismic_knn_build(seismic_index* index, uint32_t kappa, uint32_t query_cut, float heap_factor) {
    if (!index) return fail(SEISMIC_EINVAL, "knn_build: null index");
    if (!index->dev) return fail(SEISMIC_ESTATE, "knn_build: index is not on a device");
    if (kappa < 1 || kappa > kMaxRefine) return fail(SEISMIC_EINVAL, "knn_build: kappa must be in [1, %u]", kMaxRefine);
    if (!(heap_factor > 0.0f)) return fail(SEISMIC_EINVAL, "knn_build: heap_factor must be > 0");
    DeviceIndex* d = index->dev;
    DeviceGuard g(d->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "knn_build: cannot select device");
    const uint64_t n = index->h.n_docs;
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(n, 1), 65536);
    seismic_workspace* ws = nullptr;
    int rc = seismic_workspace_create(index, chunk, kappa + 1, &ws);
    if (rc) return rc;
    uint32_t *table = nullptr, *ids = nullptr;
    float* sc = nullptr;
    const size_t tbytes = std::max<size_t>((size_t)n * kappa * 4, 16);
    if (hipMalloc((void**)&table, tbytes) != hipSuccess ||
        hipMalloc((void**)&ids, (size_t)chunk * (kappa + 1) * 4) != hipSuccess ||
        hipMalloc((void**)&sc, (size_t)chunk * (kappa + 1) * 4) != hipSuccess) {
        (void)hipFree(table); (void)hipFree(ids);
        seismic_workspace_free(ws);
        return fail(SEISMIC_ENOMEM, "knn_build: device allocation failed");
    }
    seismic_search_params sp{};
    sp.k = kappa + 1;
    sp.query_cut = query_cut;
    sp.heap_factor = heap_factor;
    for (uint64_t s = 0; s < n && !rc; s += chunk) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(chunk, n - s);
        // documents [s, s + m) of the resident forward index as the queries
        seismic_csr q{m, index->nnz(), index->h.dim, 1, d->view.row_ptr + s, d->view.words};
        rc = seismic_search_batch(index, ws, &q, &sp, ids, sc, nullptr, nullptr);
        if (!rc) {
            hipLaunchKernelGGL(k_knn_finalize, dim3((m + 255) / 256), dim3(256), 0, nullptr, ids, m, (uint32_t)s, kappa,
                               table);
            if (hipGetLastError() != hipSuccess) rc = fail(SEISMIC_EHIP, "knn_build: finalize launch failed");
        }
    }
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(SEISMIC_EHIP, "knn_build: synchronize failed");
    (void)hipFree(ids);
    (void)hipFree(sc);
    seismic_workspace_free(ws);
    if (rc) {
        (void)hipFree(table);
        return rc;
    }
    std::lock_guard<std::mutex> lk(index->mu);
    (void)hipFree(d->knn);
    d->knn = table;
    d->kappa = kappa;
    return SEISMIC_OK;
}

int exact_topk(const seismic_index* index_c, const seismic_csr* queries, uint32_t k, uint32_t* out_ids,
               float* out_scores, void* stream) {
    seismic_index* index = const_cast<seismic_index*>(index_c);  // lazily extended device state
    if (!index || !queries || !out_ids || !out_scores) return fail(SEISMIC_EINVAL, "exact_topk: null argument");
    if (!index->dev) return fail(SEISMIC_ESTATE, "exact_topk: index is not on a device");
    if (k < 1 || k > SEISMIC_MAX_K) return fail(SEISMIC_EINVAL, "exact_topk: k = %u outside [1, %d]", k, SEISMIC_MAX_K);
    if (queries->dim != index->h.dim) return fail(SEISMIC_EINVAL, "exact_topk: query dim mismatch");
    DeviceIndex* d = index->dev;
    size_t smem = seismic_dev::exact_smem_bytes(k);
    if (smem > d->smem_limit) return fail(SEISMIC_EINVAL, "exact_topk: k = %u needs %zu bytes of LDS (device allows %zu)", k, smem, d->smem_limit);
    DeviceGuard g(d->device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "exact_topk: cannot select device");
    std::lock_guard<std::mutex> lk(index->mu);
    hipStream_t st = (hipStream_t)stream;
    if (!d->csc_off) {
        // column lists of the resident forward index, built on the device
        seismic_dev::DevCsc csc;
        int rc = seismic_dev::device_csc(d->view.row_ptr, d->view.words, index->h.n_docs, index->h.dim, csc, nullptr);
        if (rc) return rc;
        d->csc_off = csc.off;
        d->csc_doc = csc.doc;
        d->csc_val = csc.val;
    }
    const uint64_t* q_ptr = queries->row_ptr;
    const uint32_t* q_words = queries->words;
    const bool staged = !queries->on_device;
    if (staged) {
        int rc = validate_csr_host(queries, SEISMIC_MAX_QUERY_NNZ, "exact_topk: queries");
        if (rc) return rc;
        // the staging buffers are shared by every call on this index: wait
        // until the previous search that read them (on any stream) is done
        // before they are resized or overwritten
        if (!d->xq_done) HIP_TRY(hipEventCreateWithFlags(&d->xq_done, hipEventDisableTiming));
        else HIP_TRY(hipEventSynchronize(d->xq_done));
        rc = grow((void**)&d->xq_ptr, d->xq_rows_cap, queries->n_rows + 1, sizeof(uint64_t));
        if (!rc) rc = grow((void**)&d->xq_words, d->xq_words_cap, std::max<uint64_t>(queries->nnz, 1), sizeof(uint32_t));
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(d->xq_ptr, queries->row_ptr, (queries->n_rows + 1) * 8, hipMemcpyHostToDevice, st));
        if (queries->nnz)
            HIP_TRY(hipMemcpyAsync(d->xq_words, queries->words, queries->nnz * 4, hipMemcpyHostToDevice, st));
        q_ptr = d->xq_ptr;
        q_words = d->xq_words;
    }
    seismic_dev::ExactArgs a{};
    a.csc_off = d->csc_off;
    a.csc_doc = d->csc_doc;
    a.csc_val = d->csc_val;
    a.dim = index->h.dim;
    a.n_docs = (uint32_t)index->h.n_docs;
    a.q_ptr = q_ptr;
    a.q_words = q_words;
    a.q_nnz = queries->nnz;
    a.k = k;
    a.out_ids = out_ids;
    a.out_scores = out_scores;
    HIP_TRY(seismic_dev::launch_exact(a, (uint32_t)queries->n_rows, smem, st));
    if (staged) HIP_TRY(hipEventRecord(d->xq_done, st));
    return SEISMIC_OK;
}

}  // extern "C"

// ------------------------------------------------ search without allocation
//
// seismic_search_batch_noalloc: the query-major search with its scratch (the
// queue counter, the sanitized probe parameters and the staging of
// host-resident queries) in one file-scope device array instead of a
// workspace.  Each device holds its own copy of the array; its address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and only that address is ever handed to kernels and copies.
namespace {

constexpr size_t kNaQueueOff = 0;
constexpr size_t kNaProbeOff = 256;
constexpr size_t kNaRowsOff = kNaProbeOff + ((seismic_dev::kProbeWords * sizeof(double) + 255) & ~size_t(255));
constexpr size_t kNaRowsBytes = ((SEISMIC_NOALLOC_MAX_ROWS + 1) * sizeof(uint64_t) + 255) & ~size_t(255);
constexpr size_t kNaWordsOff = kNaRowsOff + kNaRowsBytes;
constexpr size_t kNaBytes = kNaWordsOff + (size_t)SEISMIC_NOALLOC_MAX_WORDS * sizeof(uint32_t);

static __device__ __align__(256) uint8_t scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
uint8_t* g_na_ptr[kNaMaxDevices] = {};  // device address of scratch, per device
int g_na_cus[kNaMaxDevices] = {};

// Address of this device's scratch (the device must be current).
int noalloc_setup(int device, uint8_t** ptr, int* n_cu) {
    if (device < 0 || device >= kNaMaxDevices) return fail(SEISMIC_EINVAL, "search_noalloc: device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SEISMIC_EHIP, "search_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                        hipGetErrorString(e));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, device));
        g_na_cus[device] = prop.multiProcessorCount;
        g_na_ptr[device] = (uint8_t*)p;
    }
    *ptr = g_na_ptr[device];
    *n_cu = g_na_cus[device];
    return SEISMIC_OK;
}

}  // namespace

extern "C" {

int seismic_search_batch_noalloc(const seismic_index* index, const seismic_csr* queries,
                                 const seismic_search_params* params, uint32_t* out_ids, float* out_scores,
                                 const seismic_stats* stats, void* stream) {
    if (!index || !queries || !params || !out_ids || !out_scores) return fail(SEISMIC_EINVAL, "search_noalloc: null argument");
    if (!index->dev) return fail(SEISMIC_ESTATE, "search_noalloc: index is not on a device");
    if (params->k < 1 || params->k > SEISMIC_MAX_K)
        return fail(SEISMIC_EINVAL, "search_noalloc: k = %u outside [1, %d]", params->k, SEISMIC_MAX_K);
    if (stats && stats->prefix && stats->prefix_stride < 1) return fail(SEISMIC_EINVAL, "search_noalloc: prefix_stride must be >= 1");
    if (!queries->on_device && (queries->n_rows > SEISMIC_NOALLOC_MAX_ROWS || queries->nnz > SEISMIC_NOALLOC_MAX_WORDS))
        return fail(SEISMIC_EINVAL,
                    "search_noalloc: %llu host queries with %llu nonzeros exceed the scratch (at most %d queries and %d "
                    "nonzeros; device-resident queries have no limit)",
                    (unsigned long long)queries->n_rows, (unsigned long long)queries->nnz, SEISMIC_NOALLOC_MAX_ROWS,
                    SEISMIC_NOALLOC_MAX_WORDS);
    const int device = index->dev->device;
    DeviceGuard g(device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "search_noalloc: cannot select device %d", device);
    uint8_t* ptr = nullptr;
    int n_cu = 0;
    int rc = noalloc_setup(device, &ptr, &n_cu);
    if (rc) return rc;
    // a workspace view of the scratch: no buffer of its own, no schedule
    // buffers (so the batch runs query-major), shapes as a new workspace's
    seismic_workspace ws;
    ws.index = index;
    ws.device = device;
    ws.max_queries = (uint32_t)std::min<uint64_t>(queries->n_rows, 0xFFFFFFFFull);
    ws.max_k = params->k;
    ws.n_cu = n_cu;
    ws.queue = (uint32_t*)(ptr + kNaQueueOff);
    ws.probe_w = (double*)(ptr + kNaProbeOff);
    seismic_launch_config cfg{256u, 0, 8u, 0};
    rc = check_config(&ws, &cfg);
    if (rc) return rc;
    if (queries->n_rows <= 256) {
        const seismic_launch_config wide{512u, 0, 16u, 0};
        if (check_config(&ws, &wide) == SEISMIC_OK) cfg = wide;
        clear_error();
    }
    for (int b = 0; b < kBuckets; ++b) ws.cfg[b] = cfg;
    rc = check_params(index, &ws, queries, params);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t* q_ptr = queries->row_ptr;
    const uint32_t* q_words = queries->words;
    if (!queries->on_device) {
        rc = validate_csr_host(queries, SEISMIC_MAX_QUERY_NNZ, "search_noalloc: queries");
        if (rc) return rc;
        uint64_t* d_rows = (uint64_t*)(ptr + kNaRowsOff);
        uint32_t* d_words = (uint32_t*)(ptr + kNaWordsOff);
        HIP_TRY(hipMemcpyAsync(d_rows, queries->row_ptr, (queries->n_rows + 1) * sizeof(uint64_t),
                               hipMemcpyHostToDevice, st));
        if (queries->nnz)
            HIP_TRY(hipMemcpyAsync(d_words, queries->words, queries->nnz * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        q_ptr = d_rows;
        q_words = d_words;
    }
    return launch_batch(index, &ws, q_ptr, q_words, queries->n_rows, queries->nnz, params, out_ids, out_scores, stats,
                        cfg, st);
}

}  // extern "C"
