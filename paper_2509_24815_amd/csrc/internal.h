// Internal declarations shared by the host and device parts of libseismic.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/seismic.h"

namespace seismic {

// ---------------------------------------------------------------- errors

void set_error(const char* fmt, ...);
void clear_error();

struct Error {
    int code;
    std::string msg;
};

// Returns code after recording a message; used as `return fail(SEISMIC_EINVAL, "...")`.
int fail(int code, const char* fmt, ...);

// ------------------------------------------------------------------ fp16

inline float half_to_float(uint16_t h) {
    uint32_t s = (uint32_t)(h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1Fu;
    uint32_t f = h & 0x3FFu;
    uint32_t bits;
    if (e == 0) {
        if (f == 0) bits = s;
        else {  // subnormal: normalize
            int sh = 0;
            while (!(f & 0x400u)) { f <<= 1; ++sh; }
            f &= 0x3FFu;
            bits = s | ((uint32_t)(127 - 15 - sh + 1) << 23) | (f << 13);
        }
    } else if (e == 31) {
        bits = s | 0x7F800000u | (f << 13);
    } else {
        bits = s | ((e + 112u) << 23) | (f << 13);
    }
    float out;
    std::memcpy(&out, &bits, 4);
    return out;
}

// Positive finite fp16 as an exact multiple of 2^-24.
inline uint64_t half_units24(uint16_t h) {
    uint32_t e = (h >> 10) & 0x1Fu;
    uint64_t f = h & 0x3FFu;
    return e == 0 ? f : ((1024u + f) << (e - 1));
}

inline bool half_positive_finite(uint16_t h) {
    return (h & 0x8000u) == 0 && ((h >> 10) & 0x1Fu) != 31 && (h & 0x7FFFu) != 0;
}

inline uint32_t word_term(uint32_t w) { return w & 0xFFFFu; }
inline uint16_t word_half(uint32_t w) { return (uint16_t)(w >> 16); }

// --------------------------------------------------------------- threads

// Runs fn(i, tid) for i in [0, n) on nthreads threads with dynamic chunks.
void parallel_for(int64_t n, int nthreads, int64_t chunk, const std::function<void(int64_t, int)>& fn);
int resolve_threads(int requested);

// ------------------------------------------------------------ host index

// Serialized format, version 1 (little-endian).  A 128-byte header
//   "SEISMIC\0", u32 version, u32 dim, u64 n_docs, nnz, n_blocks, n_postings,
//   n_summary, u32 lambda, u32 beta, f64 gamma, u64 seed, u32 grid bits (14),
//   u32 zero, f64 alpha (0 = fixed caps; older files hold 0 there)
// followed by 11 sections, each at a 64-byte aligned offset:
//   row_ptr u64[n_docs+1], words u32[nnz], list_off u32[dim+1],
//   blk_post_off u32[nb+1], blk_sum_off u64[nb+1], blk_m f32[nb],
//   blk_delta f32[nb], blk_centroid u32[nb], postings u32[np],
//   sum_term u16[ns], sum_code u8[ns].
constexpr uint32_t kFormatVersion = 1;
constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kGridBits = 14;  // m and the sub-interval size live on the 2^-14 grid

struct HostIndex {
    uint32_t dim = 0;
    uint64_t n_docs = 0;
    uint32_t lambda = 0, beta = 0;
    double gamma = 0.0;
    uint64_t seed = 0;
    double alpha = 0.0;  // > 0: proportional list caps (Set alpha-MSS)
    std::vector<uint64_t> row_ptr;      // forward index (Section 4.2)
    std::vector<uint32_t> words;
    std::vector<uint32_t> list_off;     // dim+1: blocks of term t are [list_off[t], list_off[t+1])
    std::vector<uint32_t> blk_post_off; // nb+1
    std::vector<uint64_t> blk_sum_off;  // nb+1
    std::vector<float> blk_m, blk_delta;
    std::vector<uint32_t> blk_centroid;
    std::vector<uint32_t> postings;
    std::vector<uint16_t> sum_term;
    std::vector<uint8_t> sum_code;

    uint64_t nnz() const { return words.size(); }
    uint64_t n_blocks() const { return blk_m.size(); }
    uint32_t max_blocks_per_list() const;
};

// Full (untruncated) inverted index: postings of term t are
// [off[t], off[t+1]) in doc-ascending order.
struct HostCSC {
    std::vector<uint64_t> off;
    std::vector<uint32_t> doc;
    std::vector<uint16_t> val;
};

int validate_csr_host(const seismic_csr* m, uint32_t max_row_nnz, const char* what);
void build_csc(const uint64_t* row_ptr, const uint32_t* words, uint64_t n_docs, uint32_t dim, int nthreads,
               HostCSC& out);
int build_host_index(const seismic_csr* docs, const seismic_build_params* p, HostIndex& out);
uint64_t list_cap(uint64_t n_full, uint32_t lambda, double alpha);
uint64_t serialized_size(const HostIndex& h);
void serialize(const HostIndex& h, uint8_t* buf);
int deserialize(const uint8_t* buf, uint64_t size, HostIndex& out);

}  // namespace seismic

// The opaque handle.  Device state lives in DeviceIndex (device.hip).
struct DeviceIndex;
struct seismic_index {
    seismic::HostIndex h;
    DeviceIndex* dev = nullptr;
    std::mutex mu;  // guards lazy device-side structures (exact search)
    // Built on a device and kept there (seismic_build_index_device): h holds
    // the parameters and the per-block arrays, but no forward index, postings
    // or summaries; their sizes are below.
    bool device_only = false;
    uint64_t dev_nnz = 0, dev_postings = 0, dev_sums = 0;
    uint64_t nnz() const { return device_only ? dev_nnz : h.nnz(); }
};

namespace seismic {
// The complete host form of a device-only index: h's arrays plus the forward
// index, postings and summaries copied back from the device (synchronous).
int download_host_index(const seismic_index* index, HostIndex& out);
// The host form to serialize: index->h itself, or a download into tmp.
int full_host_index(const seismic_index* index, HostIndex& tmp, const HostIndex** out);
}  // namespace seismic
