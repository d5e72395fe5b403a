/*
 * seismic.h - C ABI of the MI355X (gfx950) Seismic query-processing library.
 *
 * Seismic (Bruch, Nardini, Rulli, Venturini, "Efficient Sketching and Nearest
 * Neighbor Search Algorithms for Sparse Vector Sets") answers sparse maximum
 * inner product search (Definition "Sparse MIPS", Section 1.1) approximately
 * with an inverted index whose lists are truncated (Set alpha-MSS, Section
 * 3.4), clustered into blocks (Section 4.1.2) and summarized by u8-quantized
 * gamma-mass summaries (Section 4.1.3); queries are answered by Algorithm 2
 * (Section 4.5).  This library builds that index on the host, keeps it in
 * HBM and answers batches of queries with HIP kernels.
 *
 * Conventions
 *   - Every function returns 0 (SEISMIC_OK) or a negative SEISMIC_E* code;
 *     seismic_last_error() returns a thread-local message for the last
 *     failure.  No C++ exception crosses this boundary.
 *   - Sparse rows use CSR: row_ptr u64[n_rows + 1] (row_ptr[0] == 0,
 *     row_ptr[n_rows] == nnz) and one 32-bit word per nonzero: bits 0..15
 *     hold the coordinate (term id < dim), bits 16..31 the IEEE binary16
 *     value.  Terms are strictly ascending inside a row; values are finite
 *     and positive.
 *   - "device" pointers are HIP device memory on the index's device;
 *     "host" pointers are ordinary host memory.  Output buffers are always
 *     caller-owned.  Handles are library-owned and released by *_free.
 *   - stream is a hipStream_t (NULL = the legacy default stream).  Search
 *     and exact search are asynchronous on that stream.
 *   - Numerics: products of fp16 values are exact in fp32; sums are taken in
 *     fp64 and rounded once to fp32.  For values in [2^-6, 2^6] every sum is
 *     exact, so scores do not depend on summation order.
 */
#ifndef SEISMIC_H
#define SEISMIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SEISMIC_OK = 0,
    SEISMIC_EINVAL = -1,  /* invalid argument or input */
    SEISMIC_ENOMEM = -2,  /* host or device allocation failed, or a capacity was exceeded */
    SEISMIC_EHIP = -3,    /* a HIP runtime call failed */
    SEISMIC_EIO = -4,     /* file could not be read or written */
    SEISMIC_EFORMAT = -5, /* malformed or truncated serialized index */
    SEISMIC_ESTATE = -6   /* object not in the required state (e.g. index not on a device) */
};

typedef struct seismic_index seismic_index;         /* immutable after build/load */
typedef struct seismic_workspace seismic_workspace; /* per-stream scratch for search */

/* A CSR matrix of sparse rows (see Conventions).  on_device = 0: host
   pointers; 1: device pointers on the index's device. */
typedef struct {
    uint64_t n_rows;
    uint64_t nnz;
    uint32_t dim;
    uint32_t on_device;
    const uint64_t* row_ptr;
    const uint32_t* words;
} seismic_csr;

/* Index-build hyperparameters (Algorithm "Indexing with Seismic", Section
   4.4), fixed-cap form: lambda = largest values kept per coordinate (Set
   alpha-MSS with a fixed cap); beta = number of blocks of a list holding
   lambda entries (a list of n entries gets max(1, ceil(beta * n / lambda))
   blocks, empty clusters dropped); gamma = mass fraction kept by each
   block summary (gamma-MSS of the max vector, "summary" equation);
   seed keys the centroid sampling; n_threads = host threads (0 = all);
   verbose = 1 prints build phases and progress to stderr. */
typedef struct {
    uint32_t lambda;
    uint32_t beta;
    double gamma;
    uint64_t seed;
    int32_t n_threads;
    int32_t verbose;
    double alpha; /* 0: fixed caps; in (0, 1]: a column of n nonzeros keeps at most
                     min(lambda, ceil(alpha * n)) (the paper's proportional Set alpha-MSS) */
} seismic_build_params;

/* Search parameters (inputs of Algorithm 2): k results; query_cut = number
   of largest query coordinates whose lists are visited (0 = all of them),
   the fixed-size stand-in for the alpha_q-MSS of the query; query_mass =
   alpha_q > 0 selects the alpha_q-MSS itself (Definition of alpha-MSS,
   Section 3.2; Algorithm 2, first step): the largest entries (value desc,
   term asc) up to the first count whose values sum to at least alpha_q
   times the query's l1 mass, computed exactly in fp64; query_cut > 0 still
   caps that count (EINVAL for a negative or NaN query_mass); heap_factor > 0:
   a block whose summary score r satisfies r * heap_factor < heap.min (with a
   full heap) is skipped and ends its list; +INFINITY disables pruning.

   probe (device pointer, or NULL for the heap_factor rule alone): the
   SEISMIC_PROBE_WORDS bf16 parameters of the learned block probe, an
   addition to the method.  A cut list whose traversal starts with a full
   heap then evaluates exactly its blocks with probe logit >= probe_tau,
   where the logit is a 5 -> 64 -> 1 ReLU MLP of the block's features
   (r / 16, r / heap.min at the list's start, documents / 64, query
   nonzeros / 64, cut rank / 8, each rounded to bf16), evaluated exactly
   (the full definition is in the library source, probe.h).  Lists that
   start with a non-full heap keep the heap_factor rule. */
typedef struct {
    uint32_t k;
    uint32_t query_cut;
    float heap_factor;
    uint32_t flags; /* 0 or SEISMIC_SEARCH_KNN */
    const uint16_t* probe;
    double probe_tau;
    double query_mass; /* alpha_q > 0: cut = the query's alpha_q-MSS (see above); 0: query_cut alone */
} seismic_search_params;

/* flags: refine with the index's kappa-NN graph (Algorithm 2, last block;
   Section 4.3): after the traversal, S = the ids in the heap; every distinct
   neighbour of a member of S that is not in S is scored exactly and offered
   to the heap (zero scores are not results; the documents count in
   counters 3 and 4).  Needs a graph (seismic_knn_build or
   seismic_index_set_knn: ESTATE otherwise) and k * kappa <= 256 (EINVAL). */
#define SEISMIC_SEARCH_KNN 1u

#define SEISMIC_PROBE_WORDS 512 /* W1[64][5] (row = hidden unit), b1[64], w2[64], b2, zero padding */

/* Optional per-query statistics (device pointers; each may be NULL).
   prefix[q * prefix_stride + i] = number of blocks evaluated in the i-th
   visited list of query q (0 beyond the cut); counters[q * 8 + j]:
   0 summary entries of the visited lists, 1 blocks of the visited lists,
   2 blocks evaluated, 3 documents in evaluated blocks, 4 nonzeros of those
   documents, 5 prune tests made with a full heap (a probe-owned list counts
   one per block), 6 status (0 = the query row was valid, else a
   SEISMIC_QSTATUS_* bit set), 7 visited lists.
   list_hmin[q * prefix_stride + i] = smallest heap score when the i-th
   visited list starts (-1 when the heap is not full, or past the cut);
   list_term[q * prefix_stride + i] = that list's term (0xFFFFFFFF past the
   cut).  These two are the input of seismic_probe_collect. */
typedef struct {
    uint16_t* prefix;
    uint32_t prefix_stride;
    uint32_t reserved;
    uint64_t* counters;
    float* list_hmin;
    uint32_t* list_term;
} seismic_stats;

#define SEISMIC_QSTATUS_TERM_RANGE 1u /* a term id >= dim was ignored */
#define SEISMIC_QSTATUS_UNSORTED 2u   /* terms not strictly ascending */
#define SEISMIC_QSTATUS_TOO_LONG 4u   /* more than SEISMIC_MAX_QUERY_NNZ nonzeros: the rest were ignored */
#define SEISMIC_QSTATUS_BAD_VALUE 8u  /* a value was not finite and positive */

#define SEISMIC_MAX_QUERY_NNZ 1024
#define SEISMIC_MAX_K 1024

/* Message for the last failure on the calling thread ("" if none). */
const char* seismic_last_error(void);

/* Build an index on the host from host-resident documents (on_device must
   be 0).  Synchronous; the documents are copied (the forward index of
   Section 4.2 is part of the index).  EINVAL on invalid rows or
   parameters, ENOMEM on allocation failure. */
int seismic_build_index(const seismic_csr* docs, const seismic_build_params* params, seismic_index** out);

/* The same build (Algorithm "Indexing with Seismic", Section 4.4) with
   everything after input validation on HIP device `device`: the column
   lists (inverted lists before truncation) by a stable counting transpose,
   and per list the Set alpha-MSS selection, centroid sampling, K-means
   assignment, blocks, gamma-MSS summaries and quantization.  For values in
   [2^-6, 2^6] every inner product of the assignment is exact, so the index
   is byte for byte the host build's.  Lists beyond the GPU path's
   capacities (more than 1024 blocks or 2^24 kept postings in one list)
   return EINVAL: build such an index with seismic_build_index.
   Synchronous; host documents (on_device = 0); the index is returned in
   host memory like seismic_build_index's (upload it to search). */
int seismic_build_index_gpu(const seismic_csr* docs, const seismic_build_params* params, int device,
                            seismic_index** out);

/* The same build for a collection already in the memory of HIP device
   `device` (on_device = 1; rows are validated on the device as for the host
   build), and the index stays there: the result is resident on `device`
   with the plain row layout (as after seismic_index_upload with flags 0),
   ready to search, and holds no host copy of the forward index, postings or
   summaries, so a collection that fits the device but not host memory can
   be indexed.  The documents are copied into the index; the caller may free
   them once the call returns.  Device memory at the peak: the documents,
   6 bytes per nonzero of column lists, and the kept lists and summaries.
   serialize/save copy the index back to the host; upload returns ESTATE.
   The same results as seismic_build_index_gpu, byte for byte.  Lists
   beyond the capacities above return EINVAL; ENOMEM when device memory
   runs out.  Synchronous. */
int seismic_build_index_device(const seismic_csr* docs, const seismic_build_params* params, int device,
                               seismic_index** out);

/* Serialized form (format version 1, little-endian): a 128-byte header
   ("SEISMIC\0", u32 version, u32 dim, u64 n_docs, nnz, n_blocks,
   n_postings, n_summary, u32 lambda, u32 beta, f64 gamma, u64 seed, u32
   quantization grid bits, f64 alpha at offset 88), then 11 sections, each
   at a 64-byte aligned offset: row_ptr u64[n_docs+1], words u32[nnz],
   list_off u32[dim+1], blk_post_off u32[nb+1], blk_sum_off u64[nb+1],
   blk_m f32[nb], blk_delta f32[nb], blk_centroid u32[nb], postings
   u32[np], sum_term u16[ns], sum_code u8[ns].  save writes a file;
   serialize writes into a caller buffer of seismic_index_serialized_size()
   bytes (a device-built index is copied back from the device first).  EIO
   on write failure. */
int seismic_index_serialized_size(const seismic_index* index, uint64_t* bytes);
int seismic_index_serialize(const seismic_index* index, void* buf, uint64_t bytes);
int seismic_index_save(const seismic_index* index, const char* path);

/* Load a serialized index into host memory (EIO, EFORMAT on bad files). */
int seismic_index_load(const char* path, seismic_index** out);

/* out[0..7] = dim, n_docs, nnz, n_blocks, n_postings, n_summary entries,
   lambda, beta; out[8] = largest number of blocks in one list; out[9] = 1
   when the index is resident on a device (2 with block-major copies of the
   rows of every list, 3 of some lists). */
int seismic_index_info(const seismic_index* index, uint64_t out[10]);

/* Copy the index to HBM of HIP device `device` (synchronous).  Required
   before search.  ENOMEM if it does not fit, EHIP on runtime errors.
   flags: SEISMIC_UPLOAD_BLOCK_ROWS additionally stores, block after block,
   a copy of the forward rows of every block's documents (each row padded
   to 16 bytes with zero words), so that evaluating a block reads one
   contiguous run instead of scattered rows; it costs about 4 bytes per
   nonzero per posting of device memory and never changes results. */
#define SEISMIC_UPLOAD_BLOCK_ROWS 1u
int seismic_index_upload(seismic_index* index, int device, uint32_t flags);

/* Block evaluation (Algorithm 2, Section 4.5) reads the forward rows of a
   block's documents.  This stores the block-major copies that
   SEISMIC_UPLOAD_BLOCK_ROWS makes for every list for the lists
   lists[0..n_lists) (term ids, most valuable first) only, for an index
   resident on a device, uploaded or device-built, whose copies of every
   list would not fit: the longest prefix of lists[] whose copies fit in
   max_bytes of device memory is copied (16-byte padded rows, 12 bytes of
   offsets per posting and 4 bytes per block of the index).  Blocks of
   other lists keep reading their rows in place; results never change.
   Lists without postings need no copies and count as copied.  *n_copied
   (nullable) = the length of that prefix, *bytes (nullable) = the device
   memory taken; when nothing fits, nothing is stored and a later call may
   try again.  EINVAL for a term id >= dim or one given
   twice; ESTATE when the index is not resident or already has copies;
   ENOMEM when device memory runs out (nothing is kept).  Synchronous.  Not
   concurrently with searches on this index; launches made afterwards read
   the copies (graphs captured before keep reading rows in place). */
int seismic_index_copy_lists(seismic_index* index, const uint32_t* lists, uint32_t n_lists, uint64_t max_bytes,
                             uint32_t* n_copied, uint64_t* bytes);

/* Release host and device memory of the index. */
void seismic_index_free(seismic_index* index);

/* Scratch for batches of up to max_queries queries with k <= max_k on the
   index's device.  One workspace serves one stream at a time. */
int seismic_workspace_create(const seismic_index* index, uint32_t max_queries, uint32_t max_k,
                             seismic_workspace** out);
void seismic_workspace_free(seismic_workspace* ws);

/* Launch shape of the persistent search kernel held by a workspace:
   threads per workgroup (256 or 512), resident workgroups per CU
   (0 = as many as fit), the speculation window (1..32 consecutive blocks
   of a list gathered before their prune decisions are replayed in order),
   and the schedule: 0 query-major (a workgroup runs all cut lists of one
   query), 1 list-major (one launch per cut position; the items of a
   position are grouped by list, longest lists first, so that queries
   visiting the same list run together and share its blocks in the caches;
   each query's top-k is carried between positions; used when 1 <=
   query_cut <= 64, else query-major), 2 wide (for small batches: one
   workgroup per (query, cut list) scores and sorts the list's summaries;
   the first `window` blocks (1..64; twice as many, at most 64, in batches
   of at most 4 queries, which leave most of the chip idle) of every
   sorted list are cut into
   chunks of 256 documents and one workgroup per chunk scores it and keeps
   its k best documents; then one workgroup per query replays Algorithm 2's
   prune decisions in order over those stored sets, gathering any later
   block itself; used when the batch has at most 256 queries, 1 <=
   query_cut <= 32 and k <= 64, else query-major).  Results never depend on
   the shape.
   Selecting schedule 1 (set_config, or the autotuner trying it) allocates
   the workspace's list-major buffers once: about max_queries * (450 + 8 *
   max_k) bytes plus 256 bytes per index term.  Schedule 2 allocates its
   buffers once for c = min(max_queries, 256) queries and k' = min(max_k,
   64): c * 32 * (6 * sort_cap + 1028) bytes for the sorted lists and
   speculated blocks (sort_cap: the power of two at or above the index's
   longest list in blocks) plus n * (16 + 8 * k') bytes for n = min(4 * c *
   2048, max(c * 2048, 2^25 / k')) chunk items and their top-k sets.  EINVAL for
   unsupported shapes, ENOMEM if those buffers do not fit. */
typedef struct {
    uint32_t threads;
    uint32_t blocks_per_cu;
    uint32_t window;
    uint32_t schedule;
} seismic_launch_config;

/* A new workspace uses the wide schedule with 512 threads and window 32
   for batches of up to 128 queries (lowest latency), the query-major
   schedule with 512 threads and window 16 for up to 256 queries, and 256
   threads and window 8 for larger ones.  set_config applies cfg to every batch-size
   bucket (<= 128, <= 256, <= 4096, larger); get_config returns the shape
   used for a batch of n_queries queries. */
int seismic_workspace_set_config(seismic_workspace* ws, const seismic_launch_config* cfg);
int seismic_workspace_get_config(const seismic_workspace* ws, uint32_t n_queries, seismic_launch_config* cfg);
/* Search workgroups per CU that stay resident for a batch of n_queries
   queries with this k in the workspace's shape for that size: the smaller
   of the shape's blocks_per_cu (0 = no cap) and what the device fits by LDS
   and registers, as the persistent grid is sized.  LDS grows with k (16
   bytes per unit) and with the index's longest list, so a shape asking for
   3 may hold 2.  Needs the workspace's device.  EINVAL: null argument, k = 0
   or k > the workspace's max_k. */
int seismic_workspace_resident_per_cu(const seismic_workspace* ws, uint32_t n_queries, uint32_t k,
                                      uint32_t* per_cu);

/* One candidate launch shape and its mean time per search_batch call. */
typedef struct {
    seismic_launch_config cfg;
    float ms;
    uint32_t reserved;
} seismic_tune_result;

/*
 * Autotuner for the persistent search kernel.  Times seismic_search_batch
 * on this batch under every launch shape that fits the device (threads
 * 256/512 x window 1/2/4/8/16 x resident workgroups per CU 1..max, for the
 * query-major and, where they apply, list-major schedules; for the wide
 * schedule, where it applies, threads 256/512 x window 8/16/32/64), one
 * warm-up and `reps` timed calls each (HIP events on `stream`; the call
 * waits for the stream), checks that every shape returns the same ids and
 * scores (EHIP-free mismatch => ESTATE), and stores the fastest shape for
 * the batch-size bucket of queries->n_rows (buckets: <= 128, <= 256, <= 4096,
 * larger).  out_ids/out_scores are caller device buffers [n_rows * k] that
 * end up holding the results; results[0..max_results) (nullable) receive
 * every candidate's timing, *n_results their count.  queries must be
 * device resident.
 */
int seismic_autotune(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                     const seismic_search_params* params, uint32_t* out_ids, float* out_scores, uint32_t reps,
                     seismic_tune_result* results, uint32_t max_results, uint32_t* n_results, void* stream);

/*
 * Algorithm 2 (kappa = 0) for a batch of queries, asynchronously on stream.
 * out_ids [n_queries * k] u32 and out_scores [n_queries * k] f32 are device
 * buffers; each row is sorted by (score desc, id asc) and padded with
 * (0xFFFFFFFF, -INFINITY).  Host-resident queries are validated (EINVAL)
 * and copied through the workspace; device-resident queries are checked by
 * the kernel, which never reads out of bounds and reports a per-query
 * status in stats->counters.  EINVAL: bad parameters (k = 0 or > max_k,
 * heap_factor <= 0 or NaN, unknown flags, batch larger than the workspace).
 */
int seismic_search_batch(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                         const seismic_search_params* params, uint32_t* out_ids, float* out_scores,
                         const seismic_stats* stats, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as seismic_search_batch, with the same arguments, outputs and
 * errors, minus the workspace.  It calls no hipMalloc, hipFree or other
 * allocating routine: its scratch (the query queue counter, the learned
 * probe's prepared parameters and the staging of host-resident queries) is
 * a fixed device array of the library, about 4.3 MB on every device it runs
 * on, held until the process ends.  The batch always runs the query-major
 * schedule in a new workspace's shape for its size (results are those of
 * every schedule).  Limits: host-resident queries at most
 * SEISMIC_NOALLOC_MAX_ROWS rows and SEISMIC_NOALLOC_MAX_WORDS nonzeros
 * (EINVAL beyond); device-resident queries have no limit.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, or two threads) race and must be serialized by the caller.
 */
#define SEISMIC_NOALLOC_MAX_ROWS 8192
#define SEISMIC_NOALLOC_MAX_WORDS (1 << 20)
int seismic_search_batch_noalloc(const seismic_index* index, const seismic_csr* queries,
                                 const seismic_search_params* params, uint32_t* out_ids, float* out_scores,
                                 const seismic_stats* stats, void* stream);

/*
 * Exact top-k (Definition "Sparse MIPS") over the index's forward index:
 * the k documents with the largest inner product, ties by id, documents with
 * a zero score excluded, rows padded like seismic_search_batch.  The first
 * call builds a full (untruncated) inverted index of the resident forward
 * index on the device (a counting transpose; about 6 bytes per nonzero;
 * synchronous).  queries may be host or device resident; host queries are
 * validated (EINVAL) and copied on stream into staging buffers that the
 * index owns (a call first waits for the previous call's search that read
 * them).  The search itself is asynchronous on stream.  k <= SEISMIC_MAX_K.
 */
int exact_topk(const seismic_index* index, const seismic_csr* queries, uint32_t k, uint32_t* out_ids,
               float* out_scores, void* stream);

/* Free the inverted index that exact_topk built (a later exact_topk builds
 * it again).  Waits for the device to finish its work first.  A no-op when
 * there is none. */
int seismic_index_release_exact(seismic_index* index);

/* ------------------------------------------------------- kappa-NN graph
 * The graph of Section 4.3: N(u) = the kappa documents v != u with the
 * largest <u, v> (ties by id), 0xFFFFFFFF padding; table [n_docs * kappa]
 * u32, row u = N(u).  Kept on the index's device; 1 <= kappa <= 256. */

/* Approximate graph built as the paper does, with the method itself: every
 * document searched as a query (block-pruned search, k = kappa + 1,
 * query_cut, heap_factor) against the resident index, itself dropped.
 * Synchronous; replaces any previous graph. */
int seismic_knn_build(seismic_index* index, uint32_t kappa, uint32_t query_cut, float heap_factor);
/* Install a graph from host (on_device = 0) or device memory (copied). */
int seismic_index_set_knn(seismic_index* index, uint32_t kappa, const uint32_t* table, uint32_t on_device);
/* *kappa = the graph's kappa (0: none); out_host (nullable) receives the
 * table. */
int seismic_index_get_knn(const seismic_index* index, uint32_t* out_host, uint32_t* kappa);

/* ------------------------------------------------------ graph batches
 * One search launch (the kernels seismic_search_batch enqueues for
 * device-resident queries) captured into a HIP graph and replayed with
 * seismic_graph_launch.  The graph is bound to the buffers given here: the
 * queries buffer (queries->n_rows = capacity, queries->nnz = length of the
 * words buffer), the outputs and stats, the workspace and params->probe.
 * The batch size of each replay is read on the device from *n_queries_dev
 * (clamped to the capacity), so one graph serves every batch written into
 * the same buffers; row_ptr must hold n_queries + 1 valid offsets.  The
 * launch shape is the workspace's for the capacity's bucket at capture
 * time.  The captured work contains no memset nodes.  A workspace used by a
 * graph must not run other searches while the graph's replays are in
 * flight. */
typedef struct seismic_batch_graph seismic_batch_graph;
int seismic_graph_create(const seismic_index* index, seismic_workspace* ws, const seismic_csr* queries,
                         const uint32_t* n_queries_dev, const seismic_search_params* params, uint32_t* out_ids,
                         float* out_scores, const seismic_stats* stats, seismic_batch_graph** out);
int seismic_graph_launch(seismic_batch_graph* graph, void* stream);
void seismic_graph_free(seismic_batch_graph* graph);

/* ------------------------------------------------ learned block probe
 * An addition to the method (not in the paper): training on the device.
 * All buffers are caller-owned device memory; calls are asynchronous on
 * stream. */

/* Training samples from one plain search of device-resident queries: for
 * query q and its i-th cut list (i < stride) whose traversal started with a
 * full heap (list_term / list_hmin from seismic_stats of that search), every
 * block j of the list gives one sample at slot s = (q * stride + i) *
 * max_blocks + j: out_feat[s * 8 .. s * 8 + 5) = its five probe features as
 * bf16 (the other 3 words 0) and out_label[s] = 1 if the block holds one of
 * the query's exact top-k documents (exact_ids [n_rows * exact_k], e.g.
 * from exact_topk), else 0.  Slots without a sample get label 255.
 * max_blocks must be >= the largest list's block count (seismic_index_info
 * out[8]); exact_k <= 1024.  Query rows must be valid (see Conventions). */
int seismic_probe_collect(const seismic_index* index, const seismic_csr* queries, const uint32_t* list_term,
                          const float* list_hmin, uint32_t stride, const uint32_t* exact_ids, uint32_t exact_k,
                          uint32_t max_blocks, uint16_t* out_feat, uint8_t* out_label, void* stream);

typedef struct seismic_probe_trainer seismic_probe_trainer; /* device scratch for up to max_batch samples */
int seismic_probe_trainer_create(int device, uint32_t max_batch, seismic_probe_trainer** out);
void seismic_probe_trainer_free(seismic_probe_trainer* trainer);

/* Sample weights of the cross-entropy: pos_weight for label 1;
   neg_weight + neg_weight_per_doc * feature 2 (documents / 64) for label 0,
   so that a negative costs in proportion to the documents it would make the
   search score. */
typedef struct {
    float pos_weight;
    float neg_weight;
    float neg_weight_per_doc;
    uint32_t reserved;
} seismic_probe_loss;

/* Forward and backward pass over n samples (order[i] = sample index, NULL =
 * 0..n-1; samples with label 255 are skipped).  loss = sum of
 * w_s * (softplus(z_s) - y_s * z_s) with z_s the exact inference logit under
 * `weights` (SEISMIC_PROBE_WORDS bf16).  grad_out [512] fp32 = gradient sum
 * (the hidden rounding passed straight through where the pre-activation is
 * positive), accumulated in fp32 in a fixed order (deterministic);
 * stats_out [4] = loss sum, sample count, positives, weight sum.
 * n <= the trainer's max_batch. */
int seismic_probe_grad(seismic_probe_trainer* trainer, const uint16_t* feat, const uint8_t* label,
                       const uint32_t* order, uint32_t n, const seismic_probe_loss* loss, const uint16_t* weights,
                       float* grad_out, float* stats_out, void* stream);

typedef struct {
    float lr, beta1, beta2, eps;
} seismic_adam_params;

/* One Adam step on fp32 master parameters [512] with moments m, v [512]
 * from the mean gradient grad_sum / stats[1] (the outputs of
 * seismic_probe_grad); step counts from 1.  weights_out [512] receives the
 * updated parameters rounded to bf16 (nearest, ties to even); the padding
 * entries are kept at 0. */
int seismic_probe_adam(const float* grad_sum, const float* stats, float* master, float* m, float* v, uint32_t step,
                       const seismic_adam_params* params, uint16_t* weights_out, void* stream);

/* ------------------------------------------------------ serving loop
 * Continuous batching (not in the paper).  A server owns n_slots batch
 * slots, each with its own stream, search workspace, device buffers and
 * pinned staging for up to max_batch queries / max_batch_nnz nonzeros; the
 * index stays resident.  A dispatcher thread forms a batch whenever a slot
 * is free from the requests that have arrived (in submission order, up to
 * the slot's capacity), launches it (copy in, seismic_search_batch, copy
 * out) and delivers results when its event completes; batches on different
 * slots overlap on the device.  Each query's result is exactly what
 * seismic_search_batch gives for it alone (queries are independent).
 * search.probe, when set, must stay valid until the server is freed.
 *
 * Admission by scratch memory: besides a free slot, each admitted query
 * reserves its device scratch, 4 * nnz + 16 * k + 8 * L * B bytes (words,
 * result row, top-k state, and block-order buffers for its L = query_cut
 * (1024 when 0) lists of at most B blocks, B = the index's longest list),
 * from scratch_bytes; the reservation is returned when its batch completes.
 * A query whose reservation fails stays first in the queue and is admitted
 * by a later attempt: it is deferred, never dropped.
 *
 * Memory: a request's words are dropped when it is admitted and its result
 * when the caller releases its ticket (seismic_server_release); a server
 * that never releases keeps k results per query. */
typedef struct seismic_server seismic_server;
typedef struct {
    seismic_search_params search;
    uint32_t max_batch;          /* queries per batch */
    uint32_t n_slots;            /* batches in flight, 1..64 */
    uint32_t max_batch_nnz;      /* query nonzeros per batch, >= SEISMIC_MAX_QUERY_NNZ */
    uint32_t use_graphs;         /* 1: each slot's search is a captured HIP graph (seismic_graph_create),
                                    plus graphs for batches of <= 256 and <= 64 queries in the
                                    workspace's shapes for those sizes */
    seismic_launch_config launch; /* threads = 0: the workspace default */
    uint64_t scratch_bytes;      /* admission budget (see above); 0 = the slots' capacity alone;
                                    EINVAL below one query's largest reservation */
    uint32_t inject_admission_failures; /* host-forced failures for tests: the first n
                                    reservations fail as if the budget were held */
    uint32_t reserved;
} seismic_server_params;

int seismic_server_create(const seismic_index* index, const seismic_server_params* params, seismic_server** out);
/* Seconds since the server was created (its clock for not_before). */
double seismic_server_clock(const seismic_server* server);
/* Queue one query (host words, validated: EINVAL) that may be admitted from
 * server time not_before on (0 = now; must not decrease between calls).
 * *ticket identifies it; tickets count from 0 in submission order.
 * Thread-safe. */
int seismic_server_submit(seismic_server* server, const uint32_t* words, uint32_t nnz, double not_before,
                          uint64_t* ticket);
/* Queue the rows of a host CSR (validated) at once; not_before [n_rows]
 * (nullable = all now) non-decreasing; tickets are *first_ticket + row. */
int seismic_server_submit_batch(seismic_server* server, const seismic_csr* queries, const double* not_before,
                                uint64_t* first_ticket);
/* Results of tickets [first_ticket, first_ticket + n), all done (ESTATE
 * otherwise) and not released (EINVAL): ids/scores [n * k] host, latency [n]
 * seconds; each nullable. */
int seismic_server_results(seismic_server* server, uint64_t first_ticket, uint64_t n, uint32_t* ids, float* scores,
                           double* latency);
/* 1 and the result (ids/scores [k] host, nullable; latency = completion -
 * max(submission, not_before) in seconds) when done, 0 while pending, < 0 on
 * error (a failed batch stops the server). */
int seismic_server_poll(seismic_server* server, uint64_t ticket, uint32_t* ids, float* scores, double* latency);
/* Drop the results of every ticket below end_ticket (later results, polls
 * and releases of them return EINVAL).  Stops at the first ticket that is not
 * done (ESTATE); *first_held (nullable) = the first ticket still held. */
int seismic_server_release(seismic_server* server, uint64_t end_ticket, uint64_t* first_held);
/* Block until every submitted query is done (ESTATE after timeout_s). */
int seismic_server_wait_all(seismic_server* server, double timeout_s);
/* out = submitted, completed, batches launched, most queries in flight,
 * requests held (queued, in flight, or done and not released), most slots
 * busy at once, failed scratch reservations (deferred admissions), most
 * scratch bytes reserved at once. */
int seismic_server_stats(const seismic_server* server, uint64_t out[8]);
/* Stops admitting, waits for launched batches, releases everything. */
void seismic_server_free(seismic_server* server);

#ifdef __cplusplus
}
#endif

#endif /* SEISMIC_H */
