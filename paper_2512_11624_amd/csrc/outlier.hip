// Per-slice outlier terms of Sec. 2.4 applied to a rendered prediction: the
// intensity scalar sigma_i (the slice's prediction is sigma_i y) and the
// aleatoric weight omega_i = exp(rho_i), read as a per-slice likelihood
// scale:
//   masked MSE:  L = (sum_i e^{-2 rho_i} S_i + 2 n_i rho_i) / sum m,  S_i = sum m r^2
//   masked L1:   L = sum_i e^{-rho_i} S_i + n_i rho_i,             S_i = sum m |r|
// with r = sigma_i y - I and n_i = sum of the slice's mask.  A common factor
// on a subject's sigma_i trades against its amplitudes and a common shift of
// its rho_i rescales its data term against the regulariser, so the loss uses
// the per-subject centred values sigma'_i = sigma_i / geomean(sigma) and
// rho'_i = rho_i - mean(rho); the gradients with respect to log sigma and rho
// then sum to zero per subject.  Passes: per-subject means; one pass over the
// pixels (2-D grid: blocks of one slice) writing dL/dy and per-block partial
// sums; a per-slice pass folding them into S_i and the centred gradients; a
// per-subject projection; a one-block sum of the loss.  No atomics: every
// sum has a fixed order.
#include <algorithm>

#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kBlock = 256;
constexpr int kTerms = 3;   // S, n, sum dL/d(sigma y) * y

// gauge [s] = (mean log sigma, mean rho) over subject s's slices
__global__ void k_slice_gauge(const SubjectInfo* __restrict__ subj, int32_t s_n, const float* __restrict__ sigma,
                              const float* __restrict__ log_omega, float2* __restrict__ gauge) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= s_n) return;
    const int a = subj[s].s_begin, b = subj[s].s_end;
    float ls = 0.f, rr = 0.f;
    for (int i = a; i < b; ++i) {
        if (sigma) ls += logf(sigma[i]);
        if (log_omega) rr += log_omega[i];
    }
    const float inv = b > a ? 1.f / (float)(b - a) : 0.f;
    gauge[s] = make_float2(ls * inv, rr * inv);
}

__device__ inline float centred_sigma(const float* sigma, const float2* gauge, int i, int s) {
    return sigma ? sigma[i] * expf(-gauge[s].x) : 1.f;
}
__device__ inline float centred_rho(const float* log_omega, const float2* gauge, int i, int s) {
    return log_omega ? log_omega[i] - gauge[s].y : 0.f;
}

__global__ __launch_bounds__(kBlock) void k_slice_loss_pixels(
        const SliceGeo* __restrict__ geo, const float* __restrict__ pred, const float* __restrict__ target,
        const float* __restrict__ mask, const float* __restrict__ sigma, const float* __restrict__ log_omega,
        const float2* __restrict__ gauge, const float* __restrict__ msum, int32_t kind, float* __restrict__ grad,
        float* __restrict__ partial, int32_t blocks_x) {
    __shared__ float s_red[kTerms][kBlock / 64];
    const int i = blockIdx.y;
    const SliceGeo& sg = geo[i];
    const int64_t n = (int64_t)sg.H * sg.W;
    const float sg_i = centred_sigma(sigma, gauge, i, sg.subject);
    const float rho = centred_rho(log_omega, gauge, i, sg.subject);
    const float w = kind == 0 ? expf(-2.f * rho) : expf(-rho);
    const float inv_msum = (kind == 0 && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float acc[kTerms] = {0.f, 0.f, 0.f};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)blocks_x * kBlock) {
        const int64_t p = sg.pix_off + q;
        const float y = pred[p];
        const float m = mask[p];
        const float r = sg_i * y - target[p];
        float g;
        if (kind == 0) {
            acc[0] = fmaf(m * r, r, acc[0]);
            g = w * 2.f * m * r * inv_msum;
        } else {
            acc[0] = fmaf(m, fabsf(r), acc[0]);
            g = r > 0.f ? w * m : (r < 0.f ? -w * m : 0.f);
        }
        acc[1] += m;
        acc[2] = fmaf(g, y, acc[2]);
        if (grad) grad[p] = g * sg_i;
    }
    for (int e = 0; e < kTerms; ++e) {
        float v = acc[e];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) s_red[e][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < kTerms)
        partial[((int64_t)i * blocks_x + blockIdx.x) * kTerms + threadIdx.x] =
            s_red[threadIdx.x][0] + s_red[threadIdx.x][1] + s_red[threadIdx.x][2] + s_red[threadIdx.x][3];
}

// Per slice: S_i, the slice's loss, dL/dlog sigma'_i and dL/drho'_i (centred).
__global__ void k_slice_loss_slices(const float* __restrict__ partial, int32_t blocks_x, int32_t m,
                                    const SliceGeo* __restrict__ geo, const float* __restrict__ sigma,
                                    const float* __restrict__ log_omega, const float2* __restrict__ gauge,
                                    const float* __restrict__ msum, int32_t kind, float* __restrict__ slice_sums,
                                    float* __restrict__ a_sig, float* __restrict__ a_rho,
                                    float* __restrict__ slice_loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float s[kTerms] = {0.f, 0.f, 0.f};
    for (int b = 0; b < blocks_x; ++b)
        for (int e = 0; e < kTerms; ++e) s[e] += partial[((int64_t)i * blocks_x + b) * kTerms + e];
    const int subj = geo[i].subject;
    const float rho = centred_rho(log_omega, gauge, i, subj);
    float li, gr;
    if (kind == 0) {
        const float inv_msum = msum[0] > 0.f ? 1.f / msum[0] : 0.f;
        const float w = expf(-2.f * rho);
        li = (w * s[0] + 2.f * s[1] * rho) * inv_msum;
        gr = (-2.f * w * s[0] + 2.f * s[1]) * inv_msum;
    } else {
        const float w = expf(-rho);
        li = w * s[0] + s[1] * rho;
        gr = -w * s[0] + s[1];
    }
    if (slice_sums) slice_sums[i] = s[0];
    a_sig[i] = centred_sigma(sigma, gauge, i, subj) * s[2];
    a_rho[i] = gr;
    slice_loss[i] = li;
}

// Per subject: remove the mean of the centred gradients (the gauge
// directions) and map dL/dlog sigma to dL/dsigma.
__global__ void k_slice_project(const SubjectInfo* __restrict__ subj, int32_t s_n, const float* __restrict__ sigma,
                                const float* __restrict__ a_sig, const float* __restrict__ a_rho,
                                float* __restrict__ g_sigma, float* __restrict__ g_rho) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= s_n) return;
    const int a = subj[s].s_begin, b = subj[s].s_end;
    if (b <= a) return;
    float ms = 0.f, mr = 0.f;
    for (int i = a; i < b; ++i) {
        ms += a_sig[i];
        mr += a_rho[i];
    }
    ms /= (float)(b - a);
    mr /= (float)(b - a);
    for (int i = a; i < b; ++i) {
        if (g_sigma) g_sigma[i] = sigma ? (a_sig[i] - ms) / sigma[i] : a_sig[i] - ms;
        if (g_rho) g_rho[i] = a_rho[i] - mr;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_slices(const float* __restrict__ v, int32_t m,
                                                       float* __restrict__ out) {
    __shared__ float s[kBlock / 64];
    float acc = 0.f;
    for (int i = threadIdx.x; i < m; i += kBlock) acc += v[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = s[0] + s[1] + s[2] + s[3];
}

}  // namespace

int32_t slice_loss_blocks_x(int32_t max_hw) { return std::max(1, std::min((max_hw + kBlock - 1) / kBlock, 64)); }

size_t slice_loss_partial_floats(int32_t m, int32_t max_hw, int32_t s_n) {
    return (size_t)m * slice_loss_blocks_x(max_hw) * kTerms + 3 * (size_t)m + 2 * (size_t)s_n;
}

hipError_t launch_slice_loss(const SliceGeo* geo, const SubjectInfo* subj, int32_t s_n, int32_t m, int32_t max_hw,
                             const float* pred, const float* target, const float* mask, const float* sigma,
                             const float* log_omega, const float* msum, int32_t kind, float* loss, float* grad,
                             float* slice_sums, float* g_sigma, float* g_rho, float* scratch, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int bx = slice_loss_blocks_x(max_hw);
    float* partial = scratch;
    float* per_slice = scratch + (size_t)m * bx * kTerms;
    float* a_sig = per_slice + m;
    float* a_rho = a_sig + m;
    float2* gauge = (float2*)(a_rho + m);
    hipLaunchKernelGGL(k_slice_gauge, dim3((s_n + 63) / 64), dim3(64), 0, st, subj, s_n, sigma, log_omega, gauge);
    hipLaunchKernelGGL(k_slice_loss_pixels, dim3(bx, m), dim3(kBlock), 0, st, geo, pred, target, mask, sigma,
                       log_omega, (const float2*)gauge, msum, kind, grad, partial, bx);
    hipLaunchKernelGGL(k_slice_loss_slices, dim3((m + 63) / 64), dim3(64), 0, st, (const float*)partial, bx, m, geo,
                       sigma, log_omega, (const float2*)gauge, msum, kind, slice_sums, a_sig, a_rho, per_slice);
    if (g_sigma || g_rho)
        hipLaunchKernelGGL(k_slice_project, dim3((s_n + 63) / 64), dim3(64), 0, st, subj, s_n, sigma,
                           (const float*)a_sig, (const float*)a_rho, g_sigma, g_rho);
    if (loss) hipLaunchKernelGGL(k_sum_slices, dim3(1), dim3(kBlock), 0, st, (const float*)per_slice, m, loss);
    return hipGetLastError();
}

}  // namespace svr
