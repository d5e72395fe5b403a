// Host-side declarations shared by the device runtime files of libseismic.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "search_kernels.h"

#define HIP_TRY(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return seismic::fail(SEISMIC_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct DeviceIndex {
    int device = -1;
    seismic_dev::DevIdx view{};
    uint32_t sort_cap = 2;
    size_t smem_limit = 0;
    std::vector<void*> allocs;
    // full inverted index for exact search (built on first use)
    uint64_t* csc_off = nullptr;
    uint32_t* csc_doc = nullptr;
    uint16_t* csc_val = nullptr;
    // staging for host-resident queries of exact search; xq_done is recorded
    // after the last launch that reads them, on that launch's stream
    uint64_t* xq_ptr = nullptr;
    uint32_t* xq_words = nullptr;
    size_t xq_rows_cap = 0, xq_words_cap = 0;
    hipEvent_t xq_done = nullptr;
    // kappa-NN graph [n_docs * kappa] (optional)
    uint32_t* knn = nullptr;
    uint32_t kappa = 0;
    // [dim] rank of every list by block count (descending, then term):
    // the order of the list-major schedule's items
    uint32_t* term_rank = nullptr;
    // the block-major copies (view.bcopy) cover every list with postings
    bool copy_all = false;
};

// Fills d->term_rank from the list offsets (host) of the index.
int device_term_rank(DeviceIndex* d, const std::vector<uint32_t>& list_off, uint32_t dim);

// Makes a device current for the lifetime of the object.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        ok_ = hipGetDevice(&prev_) == hipSuccess && hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (ok_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = 0;
    bool ok_ = false;
};

// Grows a device buffer to at least need elements (contents are dropped).
int grow(void** p, size_t& cap, size_t need, size_t elem);

namespace seismic_dev {

// Column lists of a device-resident collection: postings of term t are
// [off[t], off[t+1]) with document ids (doc) and fp16 values (val), document
// ascending.  Device memory owned by the holder.
struct DevCsc {
    uint64_t* off = nullptr;
    uint32_t* doc = nullptr;
    uint16_t* val = nullptr;
    void release() {
        (void)hipFree(off);
        (void)hipFree(doc);
        (void)hipFree(val);
        off = nullptr;
        doc = nullptr;
        val = nullptr;
    }
};

// Builds the column lists of n_docs device rows (dim terms) on the current
// device (synchronous).  host_off, if given, receives off.  The rows must be
// valid (validate_csr_device).
int device_csc(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs, uint32_t dim, DevCsc& out,
               std::vector<uint64_t>* host_off);

// Checks device-resident rows on the current device as validate_csr_host
// does for host rows; row_max (may be NULL) receives the longest row.
int validate_csr_device(const seismic_csr* m, uint32_t max_len, const char* what, uint32_t* row_max);

}  // namespace seismic_dev
