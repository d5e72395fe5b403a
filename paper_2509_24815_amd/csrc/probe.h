// Learned block probe (an addition to the method: not in the paper).
//
// A 2-layer MLP, 5 inputs -> 64 ReLU units -> 1 logit, decides which blocks
// of a cut list are evaluated when the list's traversal starts with a full
// heap.  Its 512 parameters are stored as bf16 in the order W1[64][5]
// (row = hidden unit), b1[64], w2[64], b2, zero padding.
//
// Every step is exact, so the decision does not depend on evaluation order:
//   - a stored weight becomes 0 when NaN or |w| < 2^-12 and +-16 when
//     |w| > 16 (probe_weight);
//   - features of block j of the ci-th cut list, whose traversal starts with
//     smallest heap score h0: q(r_j / 16), q(r_j / h0), q(n_docs / 64),
//     q(n_q / 64), q(ci / 8), each ratio one fp64 operation, q = round to
//     bf16 (nearest, ties to even), 0 below 2^-8, 16 above 16;
//   - a_l = b1_l + sum_i W1[l][i] f_i; h_l = relu(a_l) rounded the same way
//     with ceiling 256; z = b2 + sum_l w2_l h_l.  All products are multiples
//     of 2^-34 and all partial sums stay below 2^19, so fp64 sums are exact.
// The list then evaluates exactly the blocks with z >= tau (in any order:
// no decision inside the list depends on the heap).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace seismic_dev {

constexpr uint32_t kProbeWords = 512;
constexpr uint32_t kProbeHidden = 64;
constexpr uint32_t kProbeIn = 5;
constexpr uint32_t kProbeB1 = kProbeHidden * kProbeIn;  // 320
constexpr uint32_t kProbeW2 = kProbeB1 + kProbeHidden;  // 384
constexpr uint32_t kProbeB2 = kProbeW2 + kProbeHidden;  // 448
constexpr uint32_t kProbeUsed = kProbeB2 + 1;           // 449

// x > 0, finite: nearest value with 8 significant bits, ties to even
// (drops the low 45 of the 52 fraction bits of the fp64 encoding).
__device__ __forceinline__ double bf16_round_pos(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    u += 0x00000FFFFFFFFFFFull + ((u >> 45) & 1ull);
    u &= ~0x00001FFFFFFFFFFFull;
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ double probe_q(double x, double lo, double hi) {
    if (!(x > 0.0)) return 0.0;
    const double y = bf16_round_pos(x);
    return y < lo ? 0.0 : (y > hi ? hi : y);
}

__device__ __forceinline__ double probe_weight(uint32_t bits16) {
    const float w = __uint_as_float(bits16 << 16);
    if (w != w || fabsf(w) < 0x1p-12f) return 0.0;
    return (double)fminf(fmaxf(w, -16.0f), 16.0f);
}

__device__ __forceinline__ void probe_features(float r, double h0, uint32_t n_docs, uint32_t n_q, uint32_t ci,
                                               double f[kProbeIn]) {
    f[0] = probe_q((double)r * 0.0625, 0x1p-8, 16.0);
    f[1] = probe_q((double)r / h0, 0x1p-8, 16.0);
    f[2] = probe_q((double)n_docs * 0.015625, 0x1p-8, 16.0);
    f[3] = probe_q((double)n_q * 0.015625, 0x1p-8, 16.0);
    f[4] = probe_q((double)ci * 0.125, 0x1p-8, 16.0);
}

// W: the sanitized parameters as fp64 (global or LDS).
__device__ __forceinline__ double probe_logit(const double* __restrict__ W, const double f[kProbeIn]) {
    double z = W[kProbeB2];
    for (uint32_t l = 0; l < kProbeHidden; ++l) {
        double a = W[kProbeB1 + l];
#pragma unroll
        for (uint32_t i = 0; i < kProbeIn; ++i) a = fma(W[l * kProbeIn + i], f[i], a);
        z = fma(W[kProbeW2 + l], probe_q(a, 0x1p-8, 256.0), z);
    }
    return z;
}

// --------------------------------------------------------------- kernels

// Training samples: one per (query, cut list, block) of lists whose
// traversal started with a full heap.
struct CollectArgs {
    DevIdx ix;
    const uint64_t* q_ptr;
    const uint32_t* q_words;
    uint64_t q_nnz;
    uint32_t nq;
    const uint32_t* list_term;  // [nq * stride]: term of the ci-th cut list (>= dim: none)
    const float* list_hmin;     // [nq * stride]: heap minimum at its start (< 0: heap not full)
    uint32_t stride;
    const uint32_t* exact_ids;  // [nq * exact_k]
    uint32_t exact_k;
    uint32_t max_blocks;        // sample slots per (query, list)
    uint16_t* out_feat;         // [nq * stride * max_blocks * 8] bf16 (5 used)
    uint8_t* out_label;         // [nq * stride * max_blocks]: 1, 0, or 255 = no sample
};

constexpr uint32_t kGradStride = 520;  // per-workgroup partials: 512 gradients, loss, count, positives, weight

struct GradArgs {
    const uint16_t* feat;   // [*, 8] bf16
    const uint8_t* label;   // 0, 1, 255 (skipped)
    const uint32_t* idx;    // sample order (NULL = 0..n-1)
    uint32_t n;
    float pos_w, neg_w, neg_w_doc;
    const double* W;        // sanitized parameters (fp64)
    float* partial;         // [grid * kGradStride]
};

constexpr uint32_t kCollectThreads = 256;
constexpr uint32_t kGradThreads = 256;

hipError_t launch_probe_prep(const uint16_t* w_bf16, double* W, hipStream_t st);
hipError_t launch_probe_collect(const CollectArgs& a, hipStream_t st);
hipError_t launch_probe_grad(const GradArgs& a, uint32_t grid, float* grad_out, float* stats_out, hipStream_t st);
hipError_t launch_probe_adam(const float* grad, const float* stats, float* master, float* m, float* v, uint32_t step,
                             float lr, float beta1, float beta2, float eps, uint16_t* w_out, hipStream_t st);

}  // namespace seismic_dev
