// dsmc_mlp.hip -- training kernels of the learned collision majorant.
//
// Network 6 -> 64 -> 64 -> 1 with ReLU (parameter order W1[64][6], b1[64],
// W2[64][64], b2[64], w3[64], b3), FP32 arithmetic, no matrix cores: the
// network is tiny and a per-sample thread keeps its 64 hidden values in
// registers while the weights sit in LDS and are read by broadcast.
//
// Training objective: mean expectile loss (Newey & Powell 1987)
//   L = (1/n_valid) sum_s |tau - 1[r_s < 0]| r_s^2,  r = label - y,
// rows with a non-finite label skipped.  The gradient is computed in
// passes: one thread per sample runs forward and backward and stores its
// activations and deltas; then the per-parameter sums over the samples are
// formed in FP64 in a fixed order (chunks of consecutive samples, then the
// chunks in order), so the result does not depend on scheduling.  Adam
// (Kingma & Ba 2015) updates in place.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/dsmc.h"

namespace {

constexpr int kIn = 6, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNp = kOffB3 + 1;
static_assert(kNp == DSMC_MLP_NPARAM, "parameter count");
constexpr int kPerSample = 4 * kH + 4;  // h1, h2, d1, d2, e, valid (+pad)
static_assert(kPerSample % 2 == 0, "the FP64 chunk sums follow the records 8-byte aligned");

__device__ __forceinline__ void load_params(const float *P, float *s) {
    for (int k = threadIdx.x; k < kNp; k += blockDim.x) s[k] = P[k];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *P, const float *x, int64_t n, float *y) {
    __shared__ float w[kNp];
    load_params(P, w);
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float in[kIn], h1[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k) in[k] = x[s * kIn + k];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = w[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kIn; ++k) a = fmaf(w[kOffW1 + o * kIn + k], in[k], a);
        h1[o] = a > 0.0f ? a : 0.0f;
    }
    float out = w[kOffB3];
    for (int o = 0; o < kH; ++o) {
        float a = w[kOffB2 + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) a = fmaf(w[kOffW2 + o * kH + i], h1[i], a);
        const float h2 = a > 0.0f ? a : 0.0f;
        out = fmaf(w[kOffW3 + o], h2, out);
    }
    y[s] = out;
}

// Forward + backward of one sample; stores h1, h2, dL/dz1, dL/dz2 (without
// the 1/n_valid factor), e = dL/dy and the loss term.
__global__ __launch_bounds__(256) void k_mlp_backward(const float *P, const float *x, const float *label,
                                                      int64_t n, float tau, float *scr) {
    __shared__ float w[kNp];
    load_params(P, w);
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float *rec = scr + s * kPerSample;
    const float lab = label[s];
    if (!isfinite(lab)) {
        for (int k = 0; k < kPerSample; ++k) rec[k] = 0.0f;
        return;
    }
    float in[kIn], h1[kH];
    uint64_t z2pos = 0ull;  // bit o set when hidden unit o of layer 2 is active
#pragma unroll
    for (int k = 0; k < kIn; ++k) in[k] = x[s * kIn + k];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = w[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kIn; ++k) a = fmaf(w[kOffW1 + o * kIn + k], in[k], a);
        h1[o] = a > 0.0f ? a : 0.0f;
        rec[o] = h1[o];
    }
    float out = w[kOffB3];
    for (int o = 0; o < kH; ++o) {
        float a = w[kOffB2 + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) a = fmaf(w[kOffW2 + o * kH + i], h1[i], a);
        const float h2 = a > 0.0f ? a : 0.0f;
        if (a > 0.0f) z2pos |= 1ull << o;
        rec[kH + o] = h2;
        out = fmaf(w[kOffW3 + o], h2, out);
    }
    const float r = lab - out;
    const float wgt = r < 0.0f ? 1.0f - tau : tau;
    const float e = -2.0f * wgt * r;  // dL/dy up to the 1/n_valid factor
    float d2[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        d2[o] = ((z2pos >> o) & 1ull) ? e * w[kOffW3 + o] : 0.0f;
        rec[3 * kH + o] = d2[o];
    }
    for (int i = 0; i < kH; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int o = 0; o < kH; ++o) a = fmaf(d2[o], w[kOffW2 + o * kH + i], a);
        rec[2 * kH + i] = h1[i] > 0.0f ? a : 0.0f;
    }
    rec[4 * kH] = e;
    rec[4 * kH + 1] = 1.0f;
    rec[4 * kH + 2] = wgt * r * r;
}

// Gradient sums in two passes, both in a fixed order.  Pass 1: block
// (bx, c) gives one thread per parameter (plus two for the loss and the
// valid count) the FP64 sum of its terms over the samples of chunk c
// (kChunk consecutive samples, ascending).  Pass 2: one thread per
// parameter adds the chunk sums in ascending chunk order and divides by the
// number of valid samples.
constexpr int kChunk = 128;
constexpr int kNq = kNp + 2;

__device__ __forceinline__ double grad_term(int q, const float *rec, const float *xs) {
    if (q < kOffB1) {
        const int o = q / kIn, k = q % kIn;
        return (double)rec[2 * kH + o] * (double)xs[k];
    }
    if (q < kOffW2) return rec[2 * kH + (q - kOffB1)];
    if (q < kOffB2) {
        const int o = (q - kOffW2) / kH, i = (q - kOffW2) % kH;
        return (double)rec[3 * kH + o] * (double)rec[i];
    }
    if (q < kOffW3) return rec[3 * kH + (q - kOffB2)];
    if (q < kOffB3) return (double)rec[4 * kH] * (double)rec[kH + (q - kOffW3)];
    if (q == kOffB3) return rec[4 * kH];
    if (q == kNp) return rec[4 * kH + 2];  // loss term
    return rec[4 * kH + 1];                // valid flag (q == kNp + 1)
}

__global__ __launch_bounds__(256) void k_mlp_partial(const float *x, int64_t n, const float *scr, double *part) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kNq) return;
    const int64_t s0 = (int64_t)blockIdx.y * kChunk;
    const int64_t s1 = s0 + kChunk < n ? s0 + kChunk : n;
    double acc = 0.0;
#pragma unroll 8
    for (int64_t s = s0; s < s1; ++s) acc += grad_term(q, scr + s * kPerSample, x + s * kIn);
    part[(int64_t)blockIdx.y * kNq + q] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_finish(const double *part, int nchunk, float *grad, float *loss) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kNp + 1) return;
    double acc = 0.0, valid = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        acc += part[(int64_t)c * kNq + q];
        valid += part[(int64_t)c * kNq + kNp + 1];
    }
    const double inv = valid > 0.0 ? 1.0 / valid : 0.0;
    if (q < kNp) grad[q] = (float)(acc * inv);
    else loss[0] = (float)(acc * inv);
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *p, const float *g, float *m, float *v, int64_t n,
                                                  float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * (gk * gk);
    m[k] = mk;
    v[k] = vk;
    p[k] = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ------------------------------------------------------------ data preparation
// Statistics of the training features over the rows with a finite label, in
// one workgroup and a fixed order (thread t takes rows t, t + 1024, ...; the
// threads' sums are added by a tree in LDS): stats[0..5] means, [6..11]
// sample standard deviations (at least 1e-6), [12] the mean label, [13] the
// number of rows.  Two passes (means, then squared deviations).
constexpr int kStatThreads = 1024;

__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kStatThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kStatThreads) void k_mlp_stats(const float *x, const float *label, int64_t n,
                                                            double *stats) {
    __shared__ double red[kStatThreads];
    double s[kIn + 2] = {};
    for (int64_t r = threadIdx.x; r < n; r += kStatThreads) {
        if (!isfinite(label[r])) continue;
#pragma unroll
        for (int k = 0; k < kIn; ++k) s[k] += (double)x[r * kIn + k];
        s[kIn] += (double)label[r];
        s[kIn + 1] += 1.0;
    }
    double tot[kIn + 2];
#pragma unroll
    for (int k = 0; k < kIn + 2; ++k) tot[k] = block_sum(s[k], red);
    const double cnt = tot[kIn + 1];
    double mean[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) mean[k] = cnt > 0.0 ? tot[k] / cnt : 0.0;
    double q[kIn] = {};
    for (int64_t r = threadIdx.x; r < n; r += kStatThreads) {
        if (!isfinite(label[r])) continue;
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            const double d = (double)x[r * kIn + k] - mean[k];
            q[k] = fma(d, d, q[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        const double v = block_sum(q[k], red);
        if (threadIdx.x == 0) {
            const double sd = cnt > 1.0 ? sqrt(v / (cnt - 1.0)) : 1.0;
            stats[k] = mean[k];
            stats[kIn + k] = sd > 1e-6 ? sd : 1e-6;
        }
    }
    if (threadIdx.x == 0) {
        stats[2 * kIn] = cnt > 0.0 ? tot[kIn] / cnt : 0.0;
        stats[2 * kIn + 1] = cnt;
    }
}

__global__ __launch_bounds__(256) void k_mlp_standardize(const float *x, int64_t n, const double *stats, float *xs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kIn) return;
    const int k = (int)(e % kIn);
    xs[e] = (float)(((double)x[e] - stats[k]) / stats[kIn + k]);
}

// A network trained on standardised inputs z = (x - m) / s takes the raw
// features after W1' = W1 / s (column-wise) and b1' = b1 - sum_k W1 m / s.
__global__ __launch_bounds__(64) void k_mlp_fold(float *P, const double *stats) {
    const int h = threadIdx.x;
    double b = (double)P[kOffB1 + h];
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        const double w = (double)P[kOffW1 + h * kIn + k] / stats[kIn + k];
        b -= w * stats[k];
        P[kOffW1 + h * kIn + k] = (float)w;
    }
    P[kOffB1 + h] = (float)b;
}

// bfloat16 of a float, rounded to nearest with ties to even (NaN stays a
// quiet NaN).
__global__ __launch_bounds__(256) void k_mlp_bf16(const float *P, int64_t n, uint16_t *bits) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t u = __float_as_uint(P[k]);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) {
        bits[k] = (uint16_t)((u >> 16) | 0x40u);
        return;
    }
    bits[k] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------- calibration
// For each margin delta_j = -0.64 + 0.01 j and each cell-size bin, the
// expected effect of the verified proposal on held-out cells (label = log2
// of the largest pair speed, bound = log2 of the exact bound, slim = log2 of
// the 65th largest r_p + r_(1)): the proposal 2^(k/64), k = ceil(64 (y +
// delta)), is verified when it is below the bound, and used when its
// verification threshold 2^(k/64) (1 - eps) is at least both the largest
// pair speed and slim; a used proposal saves cand_scale N (N - 1)
// (bound - proposal) candidates.  Costs, in candidate-equivalents: the
// network in every cell, N cost_member + cost_verify in every verified
// cell.  Sums in 2^-16 fixed point (64-bit integers, exact in any order).
constexpr double kCalFix = 65536.0;

__device__ __forceinline__ int calib_bin(double N) {
    int b = 0;
    double edge = 64.0;
    while (b < DSMC_CALIB_NBINS - 1 && N >= edge) { ++b; edge *= 2.0; }
    return b;
}

__global__ __launch_bounds__(256) void k_mlp_calibrate(const float *ypred, const float *x, const float *label,
                                                       const float *bound, const float *slim, int64_t n,
                                                       dsmc_calib_model m, unsigned long long *table) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double lab = (double)label[r], bnd = (double)bound[r];
    if (!isfinite(lab) || !isfinite(bnd)) return;
    const double N = rint(exp2((double)x[r * kIn]) * m.n_scale);
    if (N < 2.0) return;
    const int bin = calib_bin(N);
    const double sl = slim ? (double)slim[r] : -INFINITY;
    const double y = (double)ypred[r];
    const double lg1e = log2(1.0 - m.eps);
    const double cnet = m.cost_network, cver = N * m.cost_member + m.cost_verify;
    const double pairs = m.cand_scale * N * (N - 1.0);
    for (int j = 0; j < DSMC_CALIB_NDELTA; ++j) {
        const double delta = -0.64 + 0.01 * (double)j;
        double k = ceil(64.0 * (y + delta));
        k = fmin(fmax(k, -4096.0), 4096.0);
        const double gp = k / 64.0;
        unsigned long long *t = table + ((size_t)j * DSMC_CALIB_NBINS + bin) * DSMC_CALIB_FIELDS;
        double cost = cnet, gain = 0.0;
        if (gp < bnd) {
            cost += cver;
            const double gv = gp + lg1e;
            if (gv >= lab && gv >= sl) {
                gain = pairs * (exp2(bnd) - exp2(gp));
                atomicAdd(&t[2], 1ull);
            } else {
                atomicAdd(&t[3], 1ull);
            }
        }
        atomicAdd(&t[0], (unsigned long long)llrint(gain * kCalFix));
        atomicAdd(&t[1], (unsigned long long)llrint(cost * kCalFix));
    }
}

__global__ __launch_bounds__(256) void k_bf16_to_f32(const uint16_t *bits, int64_t n, float *P) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) P[k] = __uint_as_float((uint32_t)bits[k] << 16);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0ull;
}

// Scratch of the allocation-free loss-gradient call: the per-sample records
// and the FP64 chunk sums of at most DSMC_MLP_NOALLOC_MAX samples, in device
// memory that the library holds from load to process end (one copy per
// device).  Every element a call reads is written earlier in the same call,
// so nothing has to start at zero.
constexpr int64_t kNoallocFloats =
    (int64_t)DSMC_MLP_NOALLOC_MAX * kPerSample + 2 * (((int64_t)DSMC_MLP_NOALLOC_MAX + kChunk - 1) / kChunk) * kNq;
static __device__ __align__(256) float scratch[kNoallocFloats];

// Device address of `scratch` on each device, taken once per device (with
// that device current) and reused; the array's host-side name is never
// passed to a kernel.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
float *g_noalloc_ptr[kMaxDevices] = {};

dsmc_status noalloc_scratch(hipStream_t stream, float **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DSMC_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return DSMC_EINVAL;
    if (stream) {
        // the scratch address belongs to the current device: the stream must too
        hipDevice_t sdev = -1;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return DSMC_EHIP;
        if ((int)sdev != dev) return DSMC_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DSMC_EHIP;
        g_noalloc_ptr[dev] = (float *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return DSMC_OK;
}

// Loss and gradient with the given scratch (validated arguments).
dsmc_status loss_grad(const float *params, const float *x, const float *label, int64_t n, double tau, float *grad,
                      float *loss, float *scr, hipStream_t s) {
    const int nchunk = (int)((n + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, x, label, n,
                       (float)tau, scr);
    double *part = (double *)(scr + n * kPerSample);  // kPerSample is even: 8-byte aligned
    hipLaunchKernelGGL(k_mlp_partial, dim3((unsigned)((kNq + 255) / 256), (unsigned)nchunk), dim3(256), 0, s, x, n,
                       scr, part);
    hipLaunchKernelGGL(k_mlp_finish, dim3((unsigned)((kNp + 1 + 255) / 256)), dim3(256), 0, s, part, nchunk, grad,
                       loss);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

}  // namespace

extern "C" {

dsmc_status dsmc_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream) {
    if (!params || !x || !y || n < 0) return DSMC_EINVAL;
    if (n == 0) return DSMC_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       params, x, n, y);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

// per-sample records, then the FP64 chunk sums (two floats each)
int64_t dsmc_mlp_scratch_floats(int64_t n) {
    return n < 0 ? 0 : n * kPerSample + 2 * ((n + kChunk - 1) / kChunk) * (int64_t)kNq;
}

dsmc_status dsmc_mlp_loss_grad(const float *params, const float *x, const float *label, int64_t n, double tau,
                               float *grad, float *loss, float *scratch, void *stream) {
    if (!params || !x || !label || !grad || !loss || !scratch || n <= 0 || !(tau > 0.0 && tau < 1.0))
        return DSMC_EINVAL;
    if ((n + kChunk - 1) / kChunk > 65535) return DSMC_EINVAL;  // chunks are a grid dimension
    return loss_grad(params, x, label, n, tau, grad, loss, scratch, (hipStream_t)stream);
}

dsmc_status dsmc_mlp_loss_grad_noalloc(const float *params, const float *x, const float *label, int64_t n,
                                       double tau, float *grad, float *loss, void *stream) {
    if (!params || !x || !label || !grad || !loss || n <= 0 || !(tau > 0.0 && tau < 1.0)) return DSMC_EINVAL;
    if (n > DSMC_MLP_NOALLOC_MAX) return DSMC_EINVAL;
    float *scr = nullptr;
    const dsmc_status st = noalloc_scratch((hipStream_t)stream, &scr);
    if (st != DSMC_OK) return st;
    return loss_grad(params, x, label, n, tau, grad, loss, scr, (hipStream_t)stream);
}

dsmc_status dsmc_mlp_standardize(const float *x, const float *label, int64_t n, float *xs, double *stats_dev,
                                 double *stats_host, void *stream) {
    if (!x || !label || !xs || !stats_dev || n <= 0) return DSMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_stats, dim3(1), dim3(kStatThreads), 0, s, x, label, n, stats_dev);
    hipLaunchKernelGGL(k_mlp_standardize, dim3((unsigned)((n * kIn + 255) / 256)), dim3(256), 0, s, x, n, stats_dev,
                       xs);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    if (stats_host) {
        if (hipMemcpyAsync(stats_host, stats_dev, DSMC_MLP_NSTATS * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return DSMC_EHIP;
    }
    return DSMC_OK;
}

dsmc_status dsmc_mlp_fold_inputs(float *params, const double *stats_dev, void *stream) {
    if (!params || !stats_dev) return DSMC_EINVAL;
    hipLaunchKernelGGL(k_mlp_fold, dim3(1), dim3(64), 0, (hipStream_t)stream, params, stats_dev);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

dsmc_status dsmc_mlp_to_bf16(const float *params, int64_t n, uint16_t *bits, void *stream) {
    if (!params || !bits || n <= 0) return DSMC_EINVAL;
    hipLaunchKernelGGL(k_mlp_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params, n,
                       bits);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

// work: the count table, the network in FP32, the predictions
constexpr size_t kCalTableBytes = (size_t)DSMC_CALIB_NDELTA * DSMC_CALIB_NBINS * DSMC_CALIB_FIELDS * 8;
constexpr size_t kCalParamBytes = ((size_t)kNp * 4 + 255) / 256 * 256;

size_t dsmc_mlp_calib_work_bytes(int64_t n) {
    return n <= 0 ? 0 : kCalTableBytes + kCalParamBytes + (((size_t)n * 4 + 255) / 256) * 256;
}

dsmc_status dsmc_mlp_calibrate(const uint16_t *bits, const float *x, const float *label, const float *bound,
                               const float *slim, int64_t n, const dsmc_calib_model *model, void *work,
                               size_t work_bytes, double *delta_out, int32_t *min_n_out, double *table_out,
                               void *stream) {
    if (!bits || !x || !label || !bound || !model || !work || n <= 0 || !delta_out || !min_n_out)
        return DSMC_EINVAL;
    if (work_bytes < dsmc_mlp_calib_work_bytes(n) || ((uintptr_t)work & 255u)) return DSMC_EINVAL;
    if (!(model->n_scale > 0) || !(model->cand_scale >= 0) || !(model->eps >= 0 && model->eps < 0.5) ||
        !(model->cost_network >= 0) || !(model->cost_member >= 0) || !(model->cost_verify >= 0))
        return DSMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nt = (int64_t)DSMC_CALIB_NDELTA * DSMC_CALIB_NBINS * DSMC_CALIB_FIELDS;
    unsigned long long *table = (unsigned long long *)work;
    float *params = (float *)((char *)work + kCalTableBytes);
    float *ypred = (float *)((char *)work + kCalTableBytes + kCalParamBytes);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, table, nt);
    hipLaunchKernelGGL(k_bf16_to_f32, dim3((unsigned)((kNp + 255) / 256)), dim3(256), 0, s, bits, (int64_t)kNp,
                       params);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, x, n, ypred);
    hipLaunchKernelGGL(k_mlp_calibrate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ypred, x, label, bound,
                       slim, n, *model, table);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    std::vector<unsigned long long> host((size_t)nt);
    if (hipMemcpyAsync(host.data(), table, (size_t)nt * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DSMC_EHIP;
    // net saving of every (margin, gate): the bins at or above the gate use
    // the proposal, the others the exact bound directly
    double best = 0.0;
    int bj = -1, bg = DSMC_CALIB_NBINS;
    for (int j = 0; j < DSMC_CALIB_NDELTA; ++j) {
        double acc = 0.0;
        for (int g = DSMC_CALIB_NBINS - 1; g >= 0; --g) {
            const unsigned long long *t = &host[((size_t)j * DSMC_CALIB_NBINS + g) * DSMC_CALIB_FIELDS];
            acc += ((double)t[0] - (double)t[1]) / kCalFix;
            if (acc > best) { best = acc; bj = j; bg = g; }
        }
    }
    if (bj < 0) {
        // no gate repays its cost: the network is never used; the margin
        // is the one of the largest saving before costs
        double bgain = -1.0;
        for (int j = 0; j < DSMC_CALIB_NDELTA; ++j) {
            double gsum = 0.0;
            for (int g = 0; g < DSMC_CALIB_NBINS; ++g)
                gsum += (double)host[((size_t)j * DSMC_CALIB_NBINS + g) * DSMC_CALIB_FIELDS] / kCalFix;
            if (gsum > bgain) { bgain = gsum; bj = j; }
        }
        *min_n_out = INT32_MAX;
    } else {
        *min_n_out = bg == 0 ? 0 : (int32_t)(32 << bg);
    }
    *delta_out = -0.64 + 0.01 * (double)bj;
    if (table_out)
        for (int64_t i = 0; i < nt; ++i)
            table_out[i] = (i % DSMC_CALIB_FIELDS) < 2 ? (double)host[i] / kCalFix : (double)host[i];
    return DSMC_OK;
}

dsmc_status dsmc_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t n_param, int64_t t,
                          double lr, double beta1, double beta2, double eps, void *stream) {
    if (!params || !grad || !m || !v || n_param <= 0 || t < 1) return DSMC_EINVAL;
    const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n_param + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       params, grad, m, v, n_param, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                       (float)c2);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

}  // extern "C"
