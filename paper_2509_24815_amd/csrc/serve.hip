// Serving loop: continuous batching of arriving queries over a fixed set of
// batch slots.  Host code only (HIP runtime API); the search itself is
// seismic_search_batch.
//
// A slot owns everything one in-flight batch needs - a search workspace,
// device buffers for the batch's queries and results, pinned host staging
// and an event, all on its own stream - so admission is by scratch memory:
// a batch is formed only when a slot is free, from the requests that have
// arrived, in submission order, up to the slot's query and nonzero
// capacity.  Batches on different slots overlap on the device.  A
// dispatcher thread admits batches, launches them (optionally as one HIP
// graph replay per batch) and delivers finished results; callers submit and
// poll from any thread.  Admission also reserves each query's device scratch
// (query_scratch_bytes) from a budget shared by the slots, when one is set; a
// query whose reservation fails waits in the queue for the next attempt.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "device_internal.h"
#include "serve_store.h"

using namespace seismic;

namespace {

using Clock = std::chrono::steady_clock;

// Graphs for batches of up to kTinyBatch queries use the wide schedule's
// shape, larger ones (up to kSmallBatch) query-major: under load, batches
// grow and a wide batch costs more device time per query than query-major
// (8.8M index, 80k QPS: p50 2.9 ms with wide batches capped at 64, 4.0 ms
// at 128), while a lone workspace call runs wide up to 128 queries (as
// does a server without graphs: its batches run in the workspace's shape
// for their size).
constexpr uint32_t kTinyBatch = 64;    // graphs in the wide shape for up to 64 queries
constexpr uint32_t kSmallBatch = 256;  // and for up to 256 queries

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    seismic_workspace* ws = nullptr;
    uint64_t* d_ptr = nullptr;
    uint32_t* d_words = nullptr;
    uint32_t* d_ids = nullptr;
    float* d_scores = nullptr;
    uint32_t* d_nq = nullptr;    // batch size read by the captured graph
    uint32_t* h_nq = nullptr;    // pinned
    seismic_batch_graph* graph = nullptr;
    seismic_batch_graph* graph_small = nullptr;  // for batches of <= kSmallBatch queries
    seismic_batch_graph* graph_tiny = nullptr;   // for batches of <= kTinyBatch queries
    uint64_t* h_ptr = nullptr;   // pinned
    uint32_t* h_words = nullptr; // pinned
    uint32_t* h_ids = nullptr;   // pinned
    float* h_scores = nullptr;   // pinned
    std::vector<uint64_t> tickets;
    uint64_t reserved = 0;       // scratch bytes of the batch in flight
    bool busy = false;
};

}  // namespace

struct seismic_server {
    const seismic_index* index = nullptr;
    seismic_server_params p{};
    int device = -1;
    Clock::time_point t0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work;  // new requests or stop
    std::condition_variable cv_done;  // results delivered
    RequestStore store;
    ScratchBudget budget{0, 0};
    uint32_t cut_lists = 0;           // most lists a query can visit
    uint32_t max_list_blocks = 0;     // blocks of the index's longest list
    uint64_t batches = 0, max_inflight = 0, max_busy = 0;
    bool stop = false;
    int error = 0;
    std::string error_msg;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void free_slot(Slot& s) {
    if (s.graph) seismic_graph_free(s.graph);
    if (s.graph_small) seismic_graph_free(s.graph_small);
    if (s.graph_tiny) seismic_graph_free(s.graph_tiny);
    if (s.ws) seismic_workspace_free(s.ws);
    (void)hipFree(s.d_nq);
    (void)hipHostFree(s.h_nq);
    (void)hipFree(s.d_ptr);
    (void)hipFree(s.d_words);
    (void)hipFree(s.d_ids);
    (void)hipFree(s.d_scores);
    (void)hipHostFree(s.h_ptr);
    (void)hipHostFree(s.h_words);
    (void)hipHostFree(s.h_ids);
    (void)hipHostFree(s.h_scores);
    if (s.event) (void)hipEventDestroy(s.event);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot();
}

int make_slot(seismic_server* sv, Slot& s) {
    const seismic_server_params& p = sv->p;
    const size_t nq = p.max_batch, nnz = p.max_batch_nnz, nk = (size_t)p.max_batch * p.search.k;
    HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&s.event, hipEventDisableTiming));
    int rc = seismic_workspace_create(sv->index, p.max_batch, p.search.k, &s.ws);
    if (!rc && p.launch.threads) rc = seismic_workspace_set_config(s.ws, &p.launch);
    if (rc) return rc;
    if (hipMalloc((void**)&s.d_ptr, (nq + 1) * 8) != hipSuccess || hipMalloc((void**)&s.d_words, nnz * 4) != hipSuccess ||
        hipMalloc((void**)&s.d_ids, nk * 4) != hipSuccess || hipMalloc((void**)&s.d_scores, nk * 4) != hipSuccess)
        return fail(SEISMIC_ENOMEM, "server: device allocation of a slot failed");
    if (hipHostMalloc((void**)&s.h_ptr, (nq + 1) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_words, nnz * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_ids, nk * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_scores, nk * 4, hipHostMallocDefault) != hipSuccess)
        return fail(SEISMIC_ENOMEM, "server: pinned host allocation of a slot failed");
    if (p.use_graphs) {
        if (hipMalloc((void**)&s.d_nq, 4) != hipSuccess || hipHostMalloc((void**)&s.h_nq, 4, hipHostMallocDefault) != hipSuccess)
            return fail(SEISMIC_ENOMEM, "server: allocation of a slot failed");
        seismic_csr q{nq, nnz, sv->index->h.dim, 1, s.d_ptr, s.d_words};
        rc = seismic_graph_create(sv->index, s.ws, &q, s.d_nq, &p.search, s.d_ids, s.d_scores, nullptr, &s.graph);
        if (rc) return rc;
        // graphs for small and tiny batches, captured in the workspace's
        // shapes for 256 and 64 queries (unless configured: one wider
        // workgroup per query, and the wide schedule)
        if (nq > kSmallBatch) {
            seismic_csr qs{kSmallBatch, nnz, sv->index->h.dim, 1, s.d_ptr, s.d_words};
            rc = seismic_graph_create(sv->index, s.ws, &qs, s.d_nq, &p.search, s.d_ids, s.d_scores, nullptr,
                                      &s.graph_small);
            if (rc) return rc;
        }
        if (nq > kTinyBatch) {
            seismic_csr qt{kTinyBatch, nnz, sv->index->h.dim, 1, s.d_ptr, s.d_words};
            rc = seismic_graph_create(sv->index, s.ws, &qt, s.d_nq, &p.search, s.d_ids, s.d_scores, nullptr,
                                      &s.graph_tiny);
            if (rc) return rc;
        }
    }
    return SEISMIC_OK;
}

// Launch one batch on slot s (called without the lock held).
int launch(seismic_server* sv, Slot& s, uint32_t nq, uint64_t nnz) {
    const uint32_t k = sv->p.search.k;
    HIP_TRY(hipMemcpyAsync(s.d_ptr, s.h_ptr, (nq + 1) * 8, hipMemcpyHostToDevice, s.stream));
    if (nnz) HIP_TRY(hipMemcpyAsync(s.d_words, s.h_words, nnz * 4, hipMemcpyHostToDevice, s.stream));
    if (s.graph) {
        *s.h_nq = nq;
        HIP_TRY(hipMemcpyAsync(s.d_nq, s.h_nq, 4, hipMemcpyHostToDevice, s.stream));
        seismic_batch_graph* g = s.graph;
        if (nq <= kSmallBatch && s.graph_small) g = s.graph_small;
        if (nq <= kTinyBatch && s.graph_tiny) g = s.graph_tiny;
        int rc = seismic_graph_launch(g, s.stream);
        if (rc) return rc;
    } else {
        seismic_csr q{nq, nnz, sv->index->h.dim, 1, s.d_ptr, s.d_words};
        int rc = seismic_search_batch(sv->index, s.ws, &q, &sv->p.search, s.d_ids, s.d_scores, nullptr, s.stream);
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(s.h_ids, s.d_ids, (size_t)nq * k * 4, hipMemcpyDeviceToHost, s.stream));
    HIP_TRY(hipMemcpyAsync(s.h_scores, s.d_scores, (size_t)nq * k * 4, hipMemcpyDeviceToHost, s.stream));
    HIP_TRY(hipEventRecord(s.event, s.stream));
    return SEISMIC_OK;
}

void run(seismic_server* sv) {
    DeviceGuard g(sv->device);
    const uint32_t k = sv->p.search.k;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progress = false;
        // deliver finished batches
        for (Slot& s : sv->slots) {
            if (!s.busy) continue;
            lk.unlock();
            hipError_t e = hipEventQuery(s.event);
            lk.lock();
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) {
                sv->error = SEISMIC_EHIP;
                sv->error_msg = std::string("server: batch failed: ") + hipGetErrorString(e);
                sv->stop = true;
                break;
            }
            const double t = sv->now();
            for (size_t i = 0; i < s.tickets.size(); ++i)
                sv->store.deliver(s.tickets[i], s.h_ids + i * k, s.h_scores + i * k, k, t);
            sv->budget.release(s.reserved);
            s.reserved = 0;
            s.tickets.clear();
            s.busy = false;
            progress = true;
        }
        if (progress) sv->cv_done.notify_all();
        if (sv->stop) break;
        // admit arrived requests into free slots
        uint64_t inflight = 0, busy = 0;
        for (Slot& s : sv->slots) {
            if (s.busy) { inflight += s.tickets.size(); ++busy; continue; }
            const double t = sv->now();
            uint32_t nq = 0;
            uint64_t nnz = 0;
            s.h_ptr[0] = 0;
            while (sv->store.has_pending() && nq < sv->p.max_batch) {
                ServeRequest& r = sv->store.pending();
                if (r.not_before > t) break;
                if (nnz + r.words.size() > sv->p.max_batch_nnz) break;
                const uint64_t bytes = query_scratch_bytes((uint32_t)r.words.size(), k, sv->cut_lists,
                                                           sv->max_list_blocks);
                if (!sv->budget.reserve(bytes)) break;  // deferred: it stays first in the queue
                s.reserved += bytes;
                std::memcpy(s.h_words + nnz, r.words.data(), r.words.size() * 4);
                nnz += r.words.size();
                s.h_ptr[++nq] = nnz;
                s.tickets.push_back(sv->store.admit());
            }
            if (nq == 0) break;
            s.busy = true;
            ++sv->batches;
            inflight += nq;
            ++busy;
            lk.unlock();
            int rc = launch(sv, s, nq, nnz);
            lk.lock();
            if (rc) {
                sv->error = rc;
                sv->error_msg = seismic_last_error();
                sv->stop = true;
                break;
            }
            progress = true;
        }
        if (inflight > sv->max_inflight) sv->max_inflight = inflight;
        if (busy > sv->max_busy) sv->max_busy = busy;
        if (sv->stop) break;
        if (!progress) {
            // sleep until new work, the next scheduled arrival, or a short
            // poll interval for busy slots
            double wait = 50e-6;
            bool any_busy = false;
            for (Slot& s : sv->slots) any_busy |= s.busy;
            if (!any_busy) {
                if (sv->store.has_pending())
                    wait = std::max(0.0, sv->store.pending().not_before - sv->now());
                else
                    wait = 0.05;
            }
            sv->cv_work.wait_for(lk, std::chrono::duration<double>(wait));
        }
    }
    // drain: wait for launched batches before the slots are released
    lk.unlock();
    for (Slot& s : sv->slots)
        if (s.busy) (void)hipEventSynchronize(s.event);
    lk.lock();
    sv->cv_done.notify_all();
}

}  // namespace

extern "C" {

int seismic_server_create(const seismic_index* index, const seismic_server_params* params, seismic_server** out) {
    if (!index || !params || !out) return fail(SEISMIC_EINVAL, "server: null argument");
    *out = nullptr;
    if (!index->dev) return fail(SEISMIC_ESTATE, "server: index is not on a device");
    const seismic_server_params& p = *params;
    if (p.n_slots < 1 || p.n_slots > 64) return fail(SEISMIC_EINVAL, "server: n_slots must be in [1, 64]");
    if (p.max_batch < 1) return fail(SEISMIC_EINVAL, "server: max_batch must be >= 1");
    if (p.max_batch_nnz < SEISMIC_MAX_QUERY_NNZ)
        return fail(SEISMIC_EINVAL, "server: max_batch_nnz must be >= %d", SEISMIC_MAX_QUERY_NNZ);
    if (p.search.k < 1 || p.search.k > SEISMIC_MAX_K || !(p.search.heap_factor > 0.0f) ||
        (p.search.flags & ~SEISMIC_SEARCH_KNN))
        return fail(SEISMIC_EINVAL, "server: invalid search parameters");
    const uint32_t cut_lists = p.search.query_cut && p.search.query_cut < SEISMIC_MAX_QUERY_NNZ
                                   ? p.search.query_cut : SEISMIC_MAX_QUERY_NNZ;
    const uint32_t mlb = index->h.max_blocks_per_list();
    const uint64_t one = query_scratch_bytes(SEISMIC_MAX_QUERY_NNZ, p.search.k, cut_lists, mlb);
    if (p.scratch_bytes && p.scratch_bytes < one)
        return fail(SEISMIC_EINVAL, "server: scratch_bytes %llu is below one query's %llu bytes",
                    (unsigned long long)p.scratch_bytes, (unsigned long long)one);
    seismic_server* sv = new (std::nothrow) seismic_server();
    if (!sv) return fail(SEISMIC_ENOMEM, "server: host allocation failed");
    sv->index = index;
    sv->p = p;
    sv->device = index->dev->device;
    sv->budget = ScratchBudget(p.scratch_bytes, p.inject_admission_failures);
    sv->cut_lists = cut_lists;
    sv->max_list_blocks = mlb;
    DeviceGuard g(sv->device);
    sv->slots.resize(p.n_slots);
    for (Slot& s : sv->slots) {
        int rc = make_slot(sv, s);
        if (rc) {
            for (Slot& t : sv->slots) free_slot(t);
            delete sv;
            return rc;
        }
    }
    sv->t0 = Clock::now();
    try {
        sv->worker = std::thread(run, sv);
    } catch (...) {
        for (Slot& t : sv->slots) free_slot(t);
        delete sv;
        return fail(SEISMIC_ENOMEM, "server: cannot start the dispatcher thread");
    }
    *out = sv;
    return SEISMIC_OK;
}

double seismic_server_clock(const seismic_server* sv) { return sv ? sv->now() : 0.0; }

int seismic_server_submit(seismic_server* sv, const uint32_t* words, uint32_t nnz, double not_before,
                          uint64_t* ticket) {
    if (!sv || !ticket || (nnz && !words)) return fail(SEISMIC_EINVAL, "server_submit: null argument");
    if (nnz > SEISMIC_MAX_QUERY_NNZ) return fail(SEISMIC_EINVAL, "server_submit: %u nonzeros (max %d)", nnz, SEISMIC_MAX_QUERY_NNZ);
    const uint32_t dim = sv->index->h.dim;
    for (uint32_t j = 0; j < nnz; ++j) {
        const uint32_t t = word_term(words[j]);
        if (t >= dim || (j && t <= word_term(words[j - 1])) || !half_positive_finite(word_half(words[j])))
            return fail(SEISMIC_EINVAL, "server_submit: invalid query entry %u", j);
    }
    ServeRequest r;
    r.words.assign(words, words + nnz);
    const double t = sv->now();
    r.not_before = not_before;
    r.arrival = not_before > t ? not_before : t;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->error) return fail(sv->error, "%s", sv->error_msg.c_str());
    if (sv->stop) return fail(SEISMIC_ESTATE, "server_submit: server is stopping");
    if (not_before < sv->store.last_not_before())
        return fail(SEISMIC_EINVAL, "server_submit: not_before must not decrease between submissions");
    *ticket = sv->store.submit(std::move(r));
    sv->cv_work.notify_one();
    return SEISMIC_OK;
}

int seismic_server_submit_batch(seismic_server* sv, const seismic_csr* queries, const double* not_before,
                                uint64_t* first_ticket) {
    if (!sv || !queries || !first_ticket) return fail(SEISMIC_EINVAL, "server_submit_batch: null argument");
    if (queries->on_device) return fail(SEISMIC_EINVAL, "server_submit_batch: queries must be host resident");
    if (queries->dim != sv->index->h.dim) return fail(SEISMIC_EINVAL, "server_submit_batch: query dim mismatch");
    int rc = validate_csr_host(queries, SEISMIC_MAX_QUERY_NNZ, "server_submit_batch: queries");
    if (rc) return rc;
    const uint64_t n = queries->n_rows;
    for (uint64_t i = 1; i < n && not_before; ++i)
        if (not_before[i] < not_before[i - 1]) return fail(SEISMIC_EINVAL, "server_submit_batch: not_before decreases");
    std::vector<ServeRequest> add(n);
    const double t = sv->now();
    for (uint64_t i = 0; i < n; ++i) {
        ServeRequest& r = add[i];
        r.words.assign(queries->words + queries->row_ptr[i], queries->words + queries->row_ptr[i + 1]);
        r.not_before = not_before ? not_before[i] : 0.0;
        r.arrival = r.not_before > t ? r.not_before : t;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->error) return fail(sv->error, "%s", sv->error_msg.c_str());
    if (sv->stop) return fail(SEISMIC_ESTATE, "server_submit_batch: server is stopping");
    if (n && add.front().not_before < sv->store.last_not_before())
        return fail(SEISMIC_EINVAL, "server_submit_batch: not_before must not decrease between submissions");
    *first_ticket = sv->store.end();
    for (ServeRequest& r : add) sv->store.submit(std::move(r));
    sv->cv_work.notify_one();
    return SEISMIC_OK;
}

namespace {
// The request behind a ticket, or an error for a released / unknown one.
const ServeRequest* lookup(seismic_server* sv, uint64_t ticket, const char* who) {
    const ServeRequest* r = sv->store.get(ticket);
    if (!r) {
        if (ticket < sv->store.base())
            fail(SEISMIC_EINVAL, "%s: ticket %llu was released", who, (unsigned long long)ticket);
        else
            fail(SEISMIC_EINVAL, "%s: unknown ticket %llu", who, (unsigned long long)ticket);
    }
    return r;
}
}  // namespace

int seismic_server_results(seismic_server* sv, uint64_t first_ticket, uint64_t n, uint32_t* ids, float* scores,
                           double* latency) {
    if (!sv) return fail(SEISMIC_EINVAL, "server_results: null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    const uint32_t k = sv->p.search.k;
    for (uint64_t i = 0; i < n; ++i) {
        const ServeRequest* r = lookup(sv, first_ticket + i, "server_results");
        if (!r) return SEISMIC_EINVAL;
        if (!r->done) return fail(SEISMIC_ESTATE, "server_results: ticket %llu is not done", (unsigned long long)(first_ticket + i));
        if (ids) std::memcpy(ids + i * k, r->ids.data(), k * 4);
        if (scores) std::memcpy(scores + i * k, r->scores.data(), k * 4);
        if (latency) latency[i] = r->done_at - r->arrival;
    }
    return SEISMIC_OK;
}

int seismic_server_poll(seismic_server* sv, uint64_t ticket, uint32_t* ids, float* scores, double* latency) {
    if (!sv) return fail(SEISMIC_EINVAL, "server_poll: null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    const ServeRequest* r = lookup(sv, ticket, "server_poll");
    if (!r) return SEISMIC_EINVAL;
    if (!r->done) {
        if (sv->error) return fail(sv->error, "%s", sv->error_msg.c_str());
        return 0;
    }
    const uint32_t k = sv->p.search.k;
    if (ids) std::memcpy(ids, r->ids.data(), k * 4);
    if (scores) std::memcpy(scores, r->scores.data(), k * 4);
    if (latency) *latency = r->done_at - r->arrival;
    return 1;
}

int seismic_server_release(seismic_server* sv, uint64_t end_ticket, uint64_t* first_held) {
    if (!sv) return fail(SEISMIC_EINVAL, "server_release: null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (end_ticket > sv->store.end()) return fail(SEISMIC_EINVAL, "server_release: unknown tickets");
    const uint64_t b = sv->store.release(end_ticket);
    if (first_held) *first_held = b;
    if (b < end_ticket)
        return fail(SEISMIC_ESTATE, "server_release: ticket %llu is not done", (unsigned long long)b);
    return SEISMIC_OK;
}

int seismic_server_wait_all(seismic_server* sv, double timeout_s) {
    if (!sv) return fail(SEISMIC_EINVAL, "server_wait_all: null server");
    std::unique_lock<std::mutex> lk(sv->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    while (sv->store.completed() < sv->store.end() && !sv->error) {
        if (sv->cv_done.wait_until(lk, until) == std::cv_status::timeout && sv->store.completed() < sv->store.end())
            return fail(SEISMIC_ESTATE, "server_wait_all: %llu of %llu queries done after %.1f s",
                        (unsigned long long)sv->store.completed(), (unsigned long long)sv->store.end(), timeout_s);
    }
    if (sv->error) return fail(sv->error, "%s", sv->error_msg.c_str());
    return SEISMIC_OK;
}

int seismic_server_stats(const seismic_server* sv, uint64_t out[8]) {
    if (!sv || !out) return fail(SEISMIC_EINVAL, "server_stats: null argument");
    std::lock_guard<std::mutex> lk(const_cast<seismic_server*>(sv)->mu);
    out[0] = sv->store.end();
    out[1] = sv->store.completed();
    out[2] = sv->batches;
    out[3] = sv->max_inflight;
    out[4] = sv->store.held();
    out[5] = sv->max_busy;
    out[6] = sv->budget.failed();
    out[7] = sv->budget.peak();
    return SEISMIC_OK;
}

void seismic_server_free(seismic_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    DeviceGuard g(sv->device);
    for (Slot& s : sv->slots) free_slot(s);
    delete sv;
}

}  // extern "C"
