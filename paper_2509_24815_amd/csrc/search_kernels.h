// Kernel entry points and their argument blocks (host and device view).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.h"

namespace seismic_dev {

constexpr uint32_t kMaxQ = 1024;       // query nonzeros handled per query (SEISMIC_MAX_QUERY_NNZ)
constexpr uint32_t kMaxSortCap = 8192; // largest number of blocks in one list
constexpr uint32_t kMaxW = 32;         // largest speculation window (blocks)

struct SearchArgs {
    DevIdx ix;
    const uint64_t* q_ptr;
    const uint32_t* q_words;
    uint64_t q_nnz;     // length of q_words: row offsets are clamped to it
    uint32_t nq;        // queries (the capacity when nq_dev is set)
    const uint32_t* nq_dev;  // optional device word holding the batch size (<= nq), read at launch
    uint32_t k;
    uint32_t cut;
    double qmass;       // alpha_q of the query's alpha_q-MSS cut (0: query_cut alone)
    float hf;
    uint32_t sort_cap;  // power of two >= the largest list's block count
    uint32_t window;    // speculation window W in blocks, 1..kMaxW
    uint32_t* queue;    // device counter handing out queries (reset by the launch)
    uint32_t* out_ids;
    float* out_scores;
    uint16_t* prefix;
    uint32_t prefix_stride;
    uint64_t* counters;
    float* list_hmin;       // [nq * prefix_stride] heap minimum at each cut list's start (-1: not full), or NULL
    uint32_t* list_term;    // [nq * prefix_stride] term of each cut list (0xFFFFFFFF past the cut), or NULL
    const double* probe_w;  // sanitized learned-probe parameters (fp64), or NULL for the heap_factor rule
    double tau;             // probe threshold: a probe-owned list evaluates the blocks with logit >= tau
    // List-major schedule (mode == kModeList): the launch for position r
    // processes the r-th cut list of every query that has one, the items of
    // a position grouped by list (longest lists first); position 0 records
    // every query's cut lists, and each query's top-k and counters are
    // carried from one position to the next.
    uint32_t mode;          // kModeQuery or kModeList
    uint32_t pos;           // kModeList: the cut position processed
    uint32_t cmax;          // cut positions per query in ls_cut (= the query_cut, 1..kMaxPositions)
    uint16_t* ls_cut;       // [nq * cmax] cut terms (written at position 0)
    uint32_t* ls_ncut;      // [nq] cut length (written at position 0)
    const uint32_t* ls_items;  // query of every item, positions one after another
    const uint32_t* ls_seg;    // [cmax + 1] first item of each position
    float* ls_hs;           // [nq * k] carried top-k scores
    uint32_t* ls_hid;       // [nq * k] carried top-k ids
    uint32_t* ls_hn;        // [nq] carried top-k size
    uint64_t* ls_cnt;       // [nq * 6] carried counters 0..5
    // Wide schedule (mode == kModeWide, small batches): a list pass scores
    // and sorts the blocks of every (query, cut list) pair, an evaluation
    // pass scores the first `depth` blocks of each sorted list, one
    // workgroup per chunk of kWideChunk documents, keeping each chunk's k
    // best documents; then the per-query traversal makes every prune
    // decision in order, folding those stored top-k sets for the speculated
    // blocks and gathering the others itself.  Strides: cmax cut lists per
    // query, depth blocks per list.
    uint32_t depth;         // blocks speculated per cut list in batches of <= kWideTinyBatch queries
                            // (1..kWideMaxDepth; also the stride of the per-list slots)
    uint32_t depth_large;   // ... and in larger batches (<= depth)
    uint32_t wd_nt;         // threads of the traversal (its window holds at most wd_nt candidates)
    float* wd_r;            // [nq * cmax * sort_cap] summary scores in (r desc, block asc) order
    uint16_t* wd_ord;       // [nq * cmax * sort_cap] their block index within the list
    uint32_t* wd_nspec;     // [nq * cmax] speculated blocks of each cut list (a prefix of the order)
    uint4* wd_items;        // [wd_icap] evaluation items: (block, chunk, result slot, bcopy of the block)
    uint32_t wd_icap;       // item capacity
    uint32_t* wd_cnt;       // [4]: list queue, items requested, evaluation queue
    uint32_t* wd_first;     // [nq * cmax * depth] first item of each speculated block (its chunks follow)
    uint32_t* wd_docs;      // [nq * cmax * depth] documents of each speculated block
    uint64_t* wd_nnz;       // [nq * cmax * depth] and their nonzeros
    float* wd_ps;           // [wd_icap * k] top-k scores of each item's chunk (-inf padded)
    uint32_t* wd_pid;       // [wd_icap * k] and ids (0xFFFFFFFF padded)
    float* wd_lb;           // [nq] lower bound of every heap minimum after the query's first block (0: none)
    uint32_t* wd_fast;      // [nq] 1 + cut lists when the row is valid with at most kMaxSlots terms (slot of
                            // entry j = j + 1), else 0
    uint32_t* wd_cut;       // [nq * cmax] term of every cut list (rows with wd_fast set)
};

constexpr uint32_t kModeQuery = 0, kModeList = 1, kModeWide = 2;
constexpr uint32_t kMaxPositions = 64;  // largest query_cut served by the list-major schedule
constexpr uint32_t kWideMaxBatch = 256; // largest batch served by the wide schedule
constexpr uint32_t kWideMaxCut = 32;    // largest query_cut served by the wide schedule
constexpr uint32_t kWideMaxDepth = 64;  // largest speculation depth (blocks per cut list)
constexpr uint32_t kWideMaxK = 64;      // largest k served by the wide schedule
constexpr uint32_t kWideChunk = 256;    // documents per evaluation item (= its workgroup size)
constexpr uint32_t kWideTinyBatch = 4;  // batches this small speculate twice the configured depth
constexpr uint32_t kWideMetaBytes = 16 * kWideMaxDepth + 40 * kWideMaxCut;  // extra LDS of the wide traversal

// Device buffers of the list-major schedule for up to nq queries.
struct ListSched {
    uint16_t* cut = nullptr;
    uint32_t* ncut = nullptr;
    uint32_t* hist = nullptr;
    uint32_t* items = nullptr;
    uint32_t* key0 = nullptr;
    uint32_t* seg = nullptr;
    uint32_t* queues = nullptr;  // [kMaxPositions + 1]
    float* hs = nullptr;
    uint32_t* hid = nullptr;
    uint32_t* hn = nullptr;
    uint64_t* cnt = nullptr;
    const uint32_t* term_rank = nullptr;  // [dim] rank of each list by block count, descending
};

// Device buffers of the wide schedule: room for cap queries, kWideMaxCut
// cut lists of sort_cap blocks, kWideMaxDepth speculated blocks per list and
// top-k sets of k entries.
struct WideSched {
    float* r = nullptr;
    uint16_t* ord = nullptr;
    uint32_t* nspec = nullptr;
    uint4* items = nullptr;
    uint32_t* cnt = nullptr;
    uint32_t* first = nullptr;
    uint32_t* docs = nullptr;
    uint64_t* nnz = nullptr;
    float* ps = nullptr;
    uint32_t* pid = nullptr;
    float* lb = nullptr;
    uint32_t* fast = nullptr;
    uint32_t* cut = nullptr;
    uint32_t cap = 0, sort_cap = 0, k = 0, icap = 0;
};

// nt = threads per workgroup (256 or 512); grid = number of persistent workgroups.
size_t search_smem_bytes(uint32_t nt, uint32_t dim, uint32_t sort_cap, uint32_t k);
hipError_t launch_search(const SearchArgs& a, uint32_t nt, uint32_t grid, size_t smem, hipStream_t stream);
// The same search in the list-major schedule (a.cut in 1..kMaxPositions): item
// construction and one launch per cut position.
hipError_t launch_search_positions(SearchArgs a, const ListSched& ls, uint32_t nt, uint32_t grid, size_t smem,
                                hipStream_t stream);
// The same search in the wide schedule (a.cut in 1..kWideMaxCut, a.nq <=
// w.cap, a.k <= w.k, a.depth in 1..kWideMaxDepth): the list pass as a
// persistent grid of up to grid_lists workgroups of kWideListThreads
// threads (smem_lists bytes of LDS), the evaluation pass (one chunk of
// kWideChunk documents per item) of up to grid_eval workgroups of
// kWideChunk threads (smem_eval), the traversal of up to `grid` workgroups
// of nt threads (smem + kWideMetaBytes).
constexpr uint32_t kWideListThreads = 1024;
hipError_t launch_search_wide(SearchArgs a, const WideSched& w, uint32_t nt, uint32_t grid, size_t smem,
                              uint32_t grid_lists, size_t smem_lists, uint32_t grid_eval, size_t smem_eval,
                              hipStream_t stream);
int search_blocks_per_cu(uint32_t nt, size_t smem);  // resident workgroups per CU (0 on error)
// The wide evaluation pass's own LDS (k <= kWideMaxK) and residency.
size_t wide_eval_smem_bytes(uint32_t dim, uint32_t k);
int wide_eval_blocks_per_cu(size_t smem);

// Exact search over a full inverted index (term -> doc-ascending postings).
struct ExactArgs {
    const uint64_t* csc_off;  // [dim+1]
    const uint32_t* csc_doc;
    const uint16_t* csc_val;
    uint32_t dim;
    uint32_t n_docs;
    const uint64_t* q_ptr;
    const uint32_t* q_words;
    uint64_t q_nnz;
    uint32_t k;
    uint32_t* out_ids;
    float* out_scores;
};

// Refinement with the kappa-NN graph, one workgroup per query, run after
// the search on its results (ids/scores rows of k, updated in place).
struct RefineArgs {
    DevIdx ix;
    const uint64_t* q_ptr;
    const uint32_t* q_words;
    uint64_t q_nnz;
    uint32_t nq;
    const uint32_t* nq_dev;  // optional device batch size (<= nq)
    uint32_t k;
    const uint32_t* knn;     // [n_docs * kappa]
    uint32_t kappa;          // k * kappa <= kRefineThreads
    uint32_t* ids;
    float* scores;
    uint64_t* counters;      // optional [nq * 8]: documents and nonzeros added to entries 3 and 4
};

constexpr uint32_t kRefineThreads = 256;
hipError_t launch_refine(const RefineArgs& a, hipStream_t stream);

size_t exact_smem_bytes(uint32_t k);
hipError_t launch_exact(const ExactArgs& a, uint32_t nq, size_t smem, hipStream_t stream);

}  // namespace seismic_dev
