// Learned block probe: parameter preparation, training-sample collection,
// forward/backward and Adam kernels, and their C ABI entry points.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_internal.h"
#include "probe.h"

using namespace seismic;

namespace seismic_dev {

// Stored bf16 parameters -> sanitized fp64 parameters.
__global__ __launch_bounds__(kProbeWords) void k_probe_prep(const uint16_t* __restrict__ w, double* __restrict__ W) {
    const uint32_t p = threadIdx.x;
    W[p] = p < kProbeUsed ? probe_weight(w[p]) : 0.0;
}

// Binary search of term t in the sorted terms qt[0, n).
__device__ __forceinline__ double q_value(const uint16_t* qt, const double* qv, uint32_t n, uint32_t t) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (qt[mid] < t) lo = mid + 1; else hi = mid;
    }
    return (lo < n && qt[lo] == t) ? qv[lo] : 0.0;
}

// One workgroup per (query, cut-list slot).  Every slot writes all of its
// max_blocks samples (label 255 where there is no sample), so the output
// does not depend on scheduling.  Summary scores are computed exactly as
// the search computes them (exact fp64 sums, one rounding to fp32).
// Query rows must be valid (sorted, at most 1024 nonzeros used).
__global__ __launch_bounds__(kCollectThreads) void k_probe_collect(CollectArgs a) {
    __shared__ uint16_t qt[1024];
    __shared__ double qv[1024];
    __shared__ uint32_t ids[1024];
    __shared__ uint32_t nvalid;
    const uint32_t item = blockIdx.x;
    const uint32_t qi = item / a.stride, ci = item % a.stride;
    const uint32_t tid = threadIdx.x;
    const DevIdx& ix = a.ix;
    const uint32_t t = a.list_term[item];
    const float h0 = a.list_hmin[item];
    const bool have = t < ix.dim && h0 >= 0.0f;
    uint32_t nb = 0, b0 = 0;
    if (have) {
        b0 = ix.list_off[t];
        nb = min(ix.list_off[t + 1] - b0, a.max_blocks);
    }
    const uint64_t q1 = min(a.q_ptr[qi + 1], a.q_nnz), q0 = min(a.q_ptr[qi], q1);
    const uint32_t n = (uint32_t)min<uint64_t>(q1 - q0, 1024ull);
    if (tid == 0) nvalid = 0;
    __syncthreads();
    if (have) {
        uint32_t mine = 0;
        for (uint32_t j = tid; j < n; j += kCollectThreads) {
            const uint32_t w = a.q_words[q0 + j];
            const uint32_t term = w & 0xFFFFu, h = w >> 16;
            const bool ok = term < ix.dim && half_ok(h);
            qt[j] = (uint16_t)term;
            qv[j] = ok ? (double)half_bits_to_float(h) : 0.0;
            mine += ok ? 1u : 0u;
        }
        if (mine) atomicAdd(&nvalid, mine);
        for (uint32_t j = tid; j < a.exact_k; j += kCollectThreads) ids[j] = a.exact_ids[(size_t)qi * a.exact_k + j];
    }
    __syncthreads();
    const size_t base = (size_t)item * a.max_blocks;
    for (uint32_t j = tid; j < a.max_blocks; j += kCollectThreads) {
        uint4 fw = make_uint4(0, 0, 0, 0);
        uint8_t lab = 255;
        if (j < nb) {
            const uint32_t b = b0 + j;
            double A = 0.0, B = 0.0;
            for (uint64_t e = ix.blk_sum_off[b]; e < ix.blk_sum_off[b + 1]; ++e) {
                const double v = q_value(qt, qv, n, ix.sum_term[e]);
                A += v;
                B = fma(v, (double)ix.sum_code[e], B);
            }
            const float r = (float)((double)ix.blk_m[b] * A + (double)ix.blk_delta[b] * B);
            const uint32_t p0 = ix.blk_post_off[b], p1 = ix.blk_post_off[b + 1];
            lab = 0;
            for (uint32_t p = p0; p < p1 && !lab; ++p) {
                const uint32_t d = ix.postings[p];
                for (uint32_t i = 0; i < a.exact_k; ++i)
                    if (ids[i] == d) { lab = 1; break; }
            }
            double f[kProbeIn];
            probe_features(r, (double)h0, p1 - p0, nvalid, ci, f);
            uint32_t hb[kProbeIn];
#pragma unroll
            for (uint32_t i = 0; i < kProbeIn; ++i) hb[i] = __float_as_uint((float)f[i]) >> 16;  // exact: f is bf16
            fw = make_uint4(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16), hb[4], 0u);
        }
        *(uint4*)(a.out_feat + (base + j) * 8) = fw;
        a.out_label[base + j] = lab;
    }
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ __forceinline__ float softplusf(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

// Forward and backward of the weighted cross-entropy for 256 samples per
// workgroup.  The forward pass is the inference computation (exact logit);
// the backward pass runs in fp32: dz = wt * (sigmoid(z) - y), taken as
// -wt * sigmoid(-z) for y = 1 so no cancellation occurs, and the hidden
// rounding is passed straight through where a > 0.  Four groups of 64
// threads (one hidden unit per thread) each sum a quarter of the samples in
// sample order; the quarters are added in a fixed order, so the partials are
// deterministic.
__global__ __launch_bounds__(kGradThreads) void k_probe_grad(GradArgs a) {
    __shared__ double W[kProbeWords];
    __shared__ double F[kGradThreads][kProbeIn + 1];
    __shared__ float DZ[kGradThreads];
    __shared__ float part[4][kProbeHidden][8];
    __shared__ float red[kGradThreads / kWave][4];
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = tid; p < kProbeWords; p += kGradThreads) W[p] = a.W[p];
    const uint32_t s = blockIdx.x * kGradThreads + tid;
    bool valid = false, pos = false;
    double f[kProbeIn] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < a.n) {
        const uint32_t j = a.idx ? a.idx[s] : s;
        const uint8_t lab = a.label[j];
        if (lab != 255) {
            valid = true;
            pos = lab == 1;
            const uint4 fw = *(const uint4*)(a.feat + (size_t)j * 8);
            const uint32_t hb[kProbeIn] = {fw.x & 0xFFFFu, fw.x >> 16, fw.y & 0xFFFFu, fw.y >> 16, fw.z & 0xFFFFu};
#pragma unroll
            for (uint32_t i = 0; i < kProbeIn; ++i) f[i] = (double)__uint_as_float(hb[i] << 16);
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < kProbeIn; ++i) F[tid][i] = f[i];
    __syncthreads();
    float dz = 0.0f, loss = 0.0f, wt = 0.0f;
    if (valid) {
        const float z = (float)probe_logit(W, f);
        if (pos) {
            wt = a.pos_w;
            dz = -wt * sigmoidf(-z);
            loss = wt * softplusf(-z);
        } else {
            wt = a.neg_w + a.neg_w_doc * (float)f[2];
            dz = wt * sigmoidf(z);
            loss = wt * softplusf(z);
        }
    }
    DZ[tid] = dz;
    {
        float v[4] = {loss, valid ? 1.0f : 0.0f, pos ? 1.0f : 0.0f, wt};
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = wave_sum(v[c]);
        if ((tid & (kWave - 1)) == 0)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[tid / kWave][c] = v[c];
    }
    __syncthreads();
    {
        const uint32_t l = tid % kProbeHidden, quarter = tid / kProbeHidden;
        double w1[kProbeIn];
#pragma unroll
        for (uint32_t i = 0; i < kProbeIn; ++i) w1[i] = W[l * kProbeIn + i];
        const double b1 = W[kProbeB1 + l];
        const float w2 = (float)W[kProbeW2 + l];
        float g1[kProbeIn] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, gb1 = 0.0f, gw2 = 0.0f;
        const uint32_t s0 = quarter * (kGradThreads / 4), s1 = s0 + kGradThreads / 4;
        for (uint32_t t = s0; t < s1; ++t) {
            const float d = DZ[t];
            if (d == 0.0f) continue;  // not a sample (or an exactly zero contribution)
            double aa = b1;
#pragma unroll
            for (uint32_t i = 0; i < kProbeIn; ++i) aa = fma(w1[i], F[t][i], aa);
            if (aa > 0.0) {
                const float dh = d * w2;
#pragma unroll
                for (uint32_t i = 0; i < kProbeIn; ++i) g1[i] += dh * (float)F[t][i];
                gb1 += dh;
                gw2 += d * (float)probe_q(aa, 0x1p-8, 256.0);
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < kProbeIn; ++i) part[quarter][l][i] = g1[i];
        part[quarter][l][5] = gb1;
        part[quarter][l][6] = gw2;
    }
    __syncthreads();
    float* out = a.partial + (size_t)blockIdx.x * kGradStride;
    for (uint32_t p = tid; p < kProbeWords; p += kGradThreads) {
        float g = 0.0f;
        if (p < kProbeB1) {
            const uint32_t l = p / kProbeIn, i = p % kProbeIn;
            g = ((part[0][l][i] + part[1][l][i]) + part[2][l][i]) + part[3][l][i];
        } else if (p < kProbeW2) {
            const uint32_t l = p - kProbeB1;
            g = ((part[0][l][5] + part[1][l][5]) + part[2][l][5]) + part[3][l][5];
        } else if (p < kProbeB2) {
            const uint32_t l = p - kProbeW2;
            g = ((part[0][l][6] + part[1][l][6]) + part[2][l][6]) + part[3][l][6];
        } else if (p == kProbeB2) {
            for (uint32_t t = 0; t < kGradThreads; ++t) g += DZ[t];
        }
        out[p] = g;
    }
    if (tid < 4) {
        float v = 0.0f;
        for (uint32_t w = 0; w < kGradThreads / kWave; ++w) v += red[w][tid];
        out[kProbeWords + tid] = v;
    }
}

// grad_out[p] = sum over workgroups (in workgroup order) of the partials;
// stats_out = loss sum, sample count, positives, weight sum.
__global__ __launch_bounds__(1024) void k_probe_reduce(const float* __restrict__ partial, uint32_t groups,
                                                       float* __restrict__ grad_out, float* __restrict__ stats_out) {
    const uint32_t p = threadIdx.x;
    if (p >= kProbeWords + 4) return;
    float g = 0.0f;
    for (uint32_t b = 0; b < groups; ++b) g += partial[(size_t)b * kGradStride + p];
    if (p < kProbeWords) grad_out[p] = g;
    else stats_out[p - kProbeWords] = g;
}

// fp32 -> bf16 bits, nearest, ties to even (NaN -> quiet NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// One Adam step (Kingma and Ba) on the mean gradient grad / stats[1].
__global__ __launch_bounds__(kProbeWords) void k_probe_adam(const float* __restrict__ grad, const float* __restrict__ stats,
                                                            float* master, float* m, float* v, uint32_t step, float lr,
                                                            float beta1, float beta2, float eps, uint16_t* w_out) {
    const uint32_t p = threadIdx.x;
    if (p >= kProbeUsed) {
        master[p] = 0.0f;
        m[p] = 0.0f;
        v[p] = 0.0f;
        w_out[p] = 0;
        return;
    }
    const float cnt = stats[1];
    const float g = cnt > 0.0f ? grad[p] / cnt : 0.0f;
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    const float mh = mm / (1.0f - powf(beta1, (float)step));
    const float vh = vv / (1.0f - powf(beta2, (float)step));
    const float w = master[p] - lr * mh / (sqrtf(vh) + eps);
    m[p] = mm;
    v[p] = vv;
    master[p] = w;
    w_out[p] = f32_to_bf16(w);
}

hipError_t launch_probe_prep(const uint16_t* w_bf16, double* W, hipStream_t st) {
    hipLaunchKernelGGL(k_probe_prep, dim3(1), dim3(kProbeWords), 0, st, w_bf16, W);
    return hipGetLastError();
}

hipError_t launch_probe_collect(const CollectArgs& a, hipStream_t st) {
    const uint64_t items = (uint64_t)a.nq * a.stride;
    if (items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_collect, dim3((uint32_t)items), dim3(kCollectThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_probe_grad(const GradArgs& a, uint32_t grid, float* grad_out, float* stats_out, hipStream_t st) {
    if (grid) hipLaunchKernelGGL(k_probe_grad, dim3(grid), dim3(kGradThreads), 0, st, a);
    hipLaunchKernelGGL(k_probe_reduce, dim3(1), dim3(1024), 0, st, (const float*)a.partial, grid, grad_out, stats_out);
    return hipGetLastError();
}

hipError_t launch_probe_adam(const float* grad, const float* stats, float* master, float* m, float* v, uint32_t step,
                             float lr, float beta1, float beta2, float eps, uint16_t* w_out, hipStream_t st) {
    hipLaunchKernelGGL(k_probe_adam, dim3(1), dim3(kProbeWords), 0, st, grad, stats, master, m, v, step, lr, beta1,
                       beta2, eps, w_out);
    return hipGetLastError();
}

}  // namespace seismic_dev

// ------------------------------------------------------------------ C ABI

struct seismic_probe_trainer {
    int device = -1;
    uint32_t max_batch = 0;
    double* W = nullptr;       // sanitized parameters
    float* partial = nullptr;  // [groups * kGradStride]
};

extern "C" {

int seismic_probe_collect(const seismic_index* index, const seismic_csr* queries, const uint32_t* list_term,
                          const float* list_hmin, uint32_t stride, const uint32_t* exact_ids, uint32_t exact_k,
                          uint32_t max_blocks, uint16_t* out_feat, uint8_t* out_label, void* stream) {
    if (!index || !queries || !list_term || !list_hmin || !exact_ids || !out_feat || !out_label)
        return fail(SEISMIC_EINVAL, "probe_collect: null argument");
    if (!index->dev) return fail(SEISMIC_ESTATE, "probe_collect: index is not on a device");
    if (!queries->on_device) return fail(SEISMIC_EINVAL, "probe_collect: queries must be device resident");
    if (queries->dim != index->h.dim) return fail(SEISMIC_EINVAL, "probe_collect: query dim differs from the index");
    if (stride < 1) return fail(SEISMIC_EINVAL, "probe_collect: stride must be >= 1");
    if (exact_k < 1 || exact_k > 1024) return fail(SEISMIC_EINVAL, "probe_collect: exact_k must be in [1, 1024]");
    const uint32_t mb = index->h.max_blocks_per_list();
    if (max_blocks < mb) return fail(SEISMIC_EINVAL, "probe_collect: max_blocks %u < largest list (%u blocks)", max_blocks, mb);
    if (queries->n_rows * (uint64_t)stride > 0x7FFFFFFFull) return fail(SEISMIC_EINVAL, "probe_collect: batch too large");
    seismic_dev::CollectArgs a{};
    a.ix = index->dev->view;
    a.q_ptr = queries->row_ptr;
    a.q_words = queries->words;
    a.q_nnz = queries->nnz;
    a.nq = (uint32_t)queries->n_rows;
    a.list_term = list_term;
    a.list_hmin = list_hmin;
    a.stride = stride;
    a.exact_ids = exact_ids;
    a.exact_k = exact_k;
    a.max_blocks = max_blocks;
    a.out_feat = out_feat;
    a.out_label = out_label;
    DeviceGuard g(index->dev->device);
    HIP_TRY(seismic_dev::launch_probe_collect(a, (hipStream_t)stream));
    return SEISMIC_OK;
}

int seismic_probe_trainer_create(int device, uint32_t max_batch, seismic_probe_trainer** out) {
    if (!out) return fail(SEISMIC_EINVAL, "probe_trainer: null argument");
    *out = nullptr;
    if (max_batch < 1) return fail(SEISMIC_EINVAL, "probe_trainer: max_batch must be >= 1");
    DeviceGuard g(device);
    if (!g.ok()) return fail(SEISMIC_EHIP, "probe_trainer: cannot select device %d", device);
    seismic_probe_trainer* t = new (std::nothrow) seismic_probe_trainer();
    if (!t) return fail(SEISMIC_ENOMEM, "probe_trainer: host allocation failed");
    t->device = device;
    t->max_batch = max_batch;
    const size_t groups = (max_batch + seismic_dev::kGradThreads - 1) / seismic_dev::kGradThreads;
    if (hipMalloc((void**)&t->W, seismic_dev::kProbeWords * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&t->partial, std::max<size_t>(groups, 1) * seismic_dev::kGradStride * sizeof(float)) != hipSuccess) {
        (void)hipFree(t->W);
        delete t;
        return fail(SEISMIC_ENOMEM, "probe_trainer: device allocation failed");
    }
    *out = t;
    return SEISMIC_OK;
}

void seismic_probe_trainer_free(seismic_probe_trainer* t) {
    if (!t) return;
    DeviceGuard g(t->device);
    (void)hipFree(t->W);
    (void)hipFree(t->partial);
    delete t;
}

int seismic_probe_grad(seismic_probe_trainer* t, const uint16_t* feat, const uint8_t* label, const uint32_t* order,
                       uint32_t n, const seismic_probe_loss* loss, const uint16_t* weights, float* grad_out,
                       float* stats_out, void* stream) {
    if (!t || !loss || !weights || !grad_out || !stats_out || (n && (!feat || !label)))
        return fail(SEISMIC_EINVAL, "probe_grad: null argument");
    if (n > t->max_batch) return fail(SEISMIC_EINVAL, "probe_grad: %u samples exceed the trainer's batch (%u)", n, t->max_batch);
    if (!(loss->pos_weight >= 0.0f) || !(loss->neg_weight >= 0.0f) || !(loss->neg_weight_per_doc >= 0.0f))
        return fail(SEISMIC_EINVAL, "probe_grad: loss weights must be >= 0");
    DeviceGuard g(t->device);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(seismic_dev::launch_probe_prep(weights, t->W, st));
    seismic_dev::GradArgs a{};
    a.feat = feat;
    a.label = label;
    a.idx = order;
    a.n = n;
    a.pos_w = loss->pos_weight;
    a.neg_w = loss->neg_weight;
    a.neg_w_doc = loss->neg_weight_per_doc;
    a.W = t->W;
    a.partial = t->partial;
    const uint32_t groups = (n + seismic_dev::kGradThreads - 1) / seismic_dev::kGradThreads;
    HIP_TRY(seismic_dev::launch_probe_grad(a, groups, grad_out, stats_out, st));
    return SEISMIC_OK;
}

int seismic_probe_adam(const float* grad_sum, const float* stats, float* master, float* m, float* v, uint32_t step,
                       const seismic_adam_params* ap, uint16_t* weights_out, void* stream) {
    if (!grad_sum || !stats || !master || !m || !v || !ap || !weights_out)
        return fail(SEISMIC_EINVAL, "probe_adam: null argument");
    if (step < 1) return fail(SEISMIC_EINVAL, "probe_adam: step counts from 1");
    if (!(ap->lr > 0.0f) || !(ap->beta1 >= 0.0f && ap->beta1 < 1.0f) || !(ap->beta2 >= 0.0f && ap->beta2 < 1.0f) ||
        !(ap->eps > 0.0f))
        return fail(SEISMIC_EINVAL, "probe_adam: invalid hyperparameters");
    HIP_TRY(seismic_dev::launch_probe_adam(grad_sum, stats, master, m, v, step, ap->lr, ap->beta1, ap->beta2, ap->eps,
                                           weights_out, (hipStream_t)stream));
    return SEISMIC_OK;
}

}  // extern "C"
