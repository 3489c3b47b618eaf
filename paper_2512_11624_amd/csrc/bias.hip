// Multiplicative low-frequency bias field per subject (a reading of the
// paper's bias-field Gaussians, Sec. 4): subject s has K fixed broad basis
// Gaussians (centres m_k, one width w) and coefficients beta_k, and
//   b(x) = exp(sum_k beta_k phi_k(x)),  phi_k(x) = exp(-|x - m_k|^2 / (2 w^2)),
// evaluated at every pixel's world position x_p = R_i u_p + t_i under the
// slice's current pose (the field moves with the subject).  The acquired
// pixel is y'_p = b(x_p) y_p.  The adjoint of sum_p g_p y'_p gives
//   dL/dy_p = g_p b_p,  dL/dbeta_k = sum_p g_p y'_p phi_k(x_p),
//   dL/dx_p = g_p y'_p sum_k beta_k phi_k(x_p) (m_k - x_p) / w^2,
// and per slice dL/dtau = sum dL/dx_p, dL/ddelta = sum (R_i u_p) x dL/dx_p,
// dL/domega = J_l(omega)^T dL/ddelta.  Passes: pixels (2-D grid: blocks of
// one slice) writing per-block partial sums; per-slice sums of the block
// partials in block order; per-subject sums of the slices' beta terms in
// slice order, and the pose terms added to the pose gradient.  No atomics:
// every sum has a fixed order.
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kBlock = 256;

int bias_blocks_x(int32_t max_hw) {
    const int64_t b = ((int64_t)max_hw + 4 * kBlock - 1) / (4 * kBlock);
    return b < 1 ? 1 : (b > 64 ? 64 : (int)b);
}

// world position of pixel q (row-major) of slice i under its current pose
__device__ inline void pixel_world(const SliceGeo& g, const SlicePose& sp, int64_t q, float& rx, float& ry, float& rz) {
    const int r = (int)(q / g.W), k = (int)(q - (int64_t)r * g.W);
    const float u = ((float)k - 0.5f * (float)(g.W - 1)) * g.dx;
    const float v = ((float)r - 0.5f * (float)(g.H - 1)) * g.dy;
    rx = sp.R[0] * u + sp.R[1] * v;
    ry = sp.R[3] * u + sp.R[4] * v;
    rz = sp.R[6] * u + sp.R[7] * v;
}

__global__ __launch_bounds__(kBlock) void k_bias_apply(const SliceGeo* __restrict__ geo,
                                                       const SlicePose* __restrict__ pose,
                                                       const float* __restrict__ centres, float inv2w2,
                                                       const float* __restrict__ beta, int32_t K,
                                                       float* __restrict__ pred, float* __restrict__ bias,
                                                       int32_t blocks_x) {
    const int i = blockIdx.y;
    const SliceGeo& g = geo[i];
    const SlicePose& sp = pose[i];
    const int s = g.subject;
    const float* cs = centres + (size_t)s * K * 3;
    const float* bs = beta + (size_t)s * K;
    const int64_t n = (int64_t)g.H * g.W;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)blocks_x * kBlock) {
        float rx, ry, rz;
        pixel_world(g, sp, q, rx, ry, rz);
        const float x = rx + sp.t[0], y = ry + sp.t[1], z = rz + sp.t[2];
        float e = 0.f;
        for (int k = 0; k < K; ++k) {
            const float dx = cs[3 * k] - x, dy = cs[3 * k + 1] - y, dz = cs[3 * k + 2] - z;
            e = fmaf(bs[k], expf(-(dx * dx + dy * dy + dz * dz) * inv2w2), e);
        }
        const float b = expf(e);
        const int64_t p = g.pix_off + q;
        pred[p] *= b;
        if (bias) bias[p] = b;
    }
}

// Per block: K beta terms, then dL/dtau (3) and dL/ddelta (3), to partial
// [slice][block][K + 6]; grad_pred (dL/dy') becomes dL/dy in place.  KM >= K
// bounds the basis loop at compile time so the sums stay in registers.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_bias_pixels(const SliceGeo* __restrict__ geo,
                                                        const SlicePose* __restrict__ pose,
                                                        const float* __restrict__ centres, float inv2w2,
                                                        const float* __restrict__ beta, int32_t K,
                                                        const float* __restrict__ pred_biased,
                                                        const float* __restrict__ bias, float* __restrict__ grad,
                                                        float* __restrict__ partial, int32_t blocks_x) {
    constexpr int NW = kBlock / 64;
    __shared__ float s_red[KM + 6][NW];
    const int i = blockIdx.y;
    const SliceGeo& g = geo[i];
    const SlicePose& sp = pose[i];
    const int s = g.subject;
    const float* cs = centres + (size_t)s * K * 3;
    const float* bs = beta + (size_t)s * K;
    const int64_t n = (int64_t)g.H * g.W;
    const float twice = 2.f * inv2w2;   // 1 / w^2
    float acc[KM + 6];
#pragma unroll
    for (int k = 0; k < KM + 6; ++k) acc[k] = 0.f;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)blocks_x * kBlock) {
        float rx, ry, rz;
        pixel_world(g, sp, q, rx, ry, rz);
        const float x = rx + sp.t[0], y = ry + sp.t[1], z = rz + sp.t[2];
        const int64_t p = g.pix_off + q;
        const float gv = grad[p];
        const float w = gv * pred_biased[p];   // g y'
        grad[p] = gv * bias[p];
        float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < K) {
                const float dx = cs[3 * k] - x, dy = cs[3 * k + 1] - y, dz = cs[3 * k + 2] - z;
                const float ph = expf(-(dx * dx + dy * dy + dz * dz) * inv2w2);
                acc[k] = fmaf(w, ph, acc[k]);
                const float c = w * bs[k] * ph * twice;
                gx = fmaf(c, dx, gx);
                gy = fmaf(c, dy, gy);
                gz = fmaf(c, dz, gz);
            }
        }
        acc[KM] += gx;
        acc[KM + 1] += gy;
        acc[KM + 2] += gz;
        // (R u) x dL/dx
        acc[KM + 3] += ry * gz - rz * gy;
        acc[KM + 4] += rz * gx - rx * gz;
        acc[KM + 5] += rx * gy - ry * gx;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < KM + 6; ++e) {
        if (e < K || e >= KM) {
            float v = acc[e];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) s_red[e][wv] = v;
        }
    }
    __syncthreads();
    const int nt = K + 6;
    for (int e = threadIdx.x; e < nt; e += kBlock) {
        const int src = e < K ? e : KM + (e - K);
        float v = 0.f;
        for (int q2 = 0; q2 < NW; ++q2) v += s_red[src][q2];
        partial[((size_t)i * blocks_x + blockIdx.x) * nt + e] = v;
    }
}

// per slice: sums of its block partials in block order -> terms [slice][K + 6]
__global__ void k_bias_slices(const float* __restrict__ partial, int32_t m, int32_t K, int32_t blocks_x,
                              float* __restrict__ terms) {
    const int nt = K + 6;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * nt) return;
    const int i = (int)(t / nt), e = (int)(t - (int64_t)i * nt);
    float v = 0.f;
    for (int b = 0; b < blocks_x; ++b) v += partial[((size_t)i * blocks_x + b) * nt + e];
    terms[t] = v;
}

// per subject and basis: sum of its slices' beta terms in slice order
__global__ void k_bias_beta(const float* __restrict__ terms, const SubjectInfo* __restrict__ subj, int32_t s_n,
                            int32_t K, float* __restrict__ g_beta) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)s_n * K) return;
    const int s = (int)(t / K), k = (int)(t - (int64_t)s * K);
    float v = 0.f;
    for (int i = subj[s].s_begin; i < subj[s].s_end; ++i) v += terms[(size_t)i * (K + 6) + k];
    g_beta[t] = v;
}

// per slice: dL/dtau and J_l(omega)^T dL/ddelta added to g_pose [M, 6]
__global__ void k_bias_pose(const float* __restrict__ terms, const SlicePose* __restrict__ pose, int32_t m,
                            int32_t K, float* __restrict__ g_pose) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float* tm = terms + (size_t)i * (K + 6) + K;
    const float wx = pose[i].w[0], wy = pose[i].w[1], wz = pose[i].w[2];
    const float th2 = wx * wx + wy * wy + wz * wz, th = sqrtf(th2);
    float A, B;  // J_l = I + A [w]x + B [w]x^2
    if (th < 1e-3f) {
        A = 0.5f - th2 * (1.f / 24.f);
        B = 1.f / 6.f - th2 * (1.f / 120.f);
    } else {
        A = (1.f - cosf(th)) / th2;
        B = (th - sinf(th)) / (th2 * th);
    }
    const float d0 = tm[3], d1 = tm[4], d2 = tm[5];
    // J_l^T d = d - A (w x d) + B (w x (w x d))
    const float c0 = wy * d2 - wz * d1, c1 = wz * d0 - wx * d2, c2 = wx * d1 - wy * d0;
    const float e0 = wy * c2 - wz * c1, e1 = wz * c0 - wx * c2, e2 = wx * c1 - wy * c0;
    g_pose[6 * i] += d0 - A * c0 + B * e0;
    g_pose[6 * i + 1] += d1 - A * c1 + B * e1;
    g_pose[6 * i + 2] += d2 - A * c2 + B * e2;
    g_pose[6 * i + 3] += tm[0];
    g_pose[6 * i + 4] += tm[1];
    g_pose[6 * i + 5] += tm[2];
}

}  // namespace

size_t bias_scratch_floats(int32_t m, int32_t max_hw, int32_t K) {
    return (size_t)m * bias_blocks_x(max_hw) * (K + 6) + (size_t)m * (K + 6);
}

hipError_t launch_bias_apply(const SliceGeo* geo, const SlicePose* pose, int32_t m, int32_t max_hw,
                             const float* centres, float width, const float* beta, int32_t K, float* pred,
                             float* bias, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int bx = bias_blocks_x(max_hw);
    hipLaunchKernelGGL(k_bias_apply, dim3(bx, m), dim3(kBlock), 0, st, geo, pose, centres,
                       0.5f / (width * width), beta, K, pred, bias, bx);
    return hipGetLastError();
}

hipError_t launch_bias_backward(const SliceGeo* geo, const SlicePose* pose, const SubjectInfo* subj, int32_t s_n,
                                int32_t m, int32_t max_hw, const float* centres, float width, const float* beta,
                                int32_t K, const float* pred_biased, const float* bias, float* grad,
                                float* g_beta, float* g_pose, float* scratch, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int bx = bias_blocks_x(max_hw);
    float* partial = scratch;
    float* terms = scratch + (size_t)m * bx * (K + 6);
    const float inv2w2 = 0.5f / (width * width);
    if (K <= 8)
        hipLaunchKernelGGL(k_bias_pixels<8>, dim3(bx, m), dim3(kBlock), 0, st, geo, pose, centres, inv2w2, beta, K,
                           pred_biased, bias, grad, partial, bx);
    else if (K <= 32)
        hipLaunchKernelGGL(k_bias_pixels<32>, dim3(bx, m), dim3(kBlock), 0, st, geo, pose, centres, inv2w2, beta, K,
                           pred_biased, bias, grad, partial, bx);
    else if (K <= kBiasMaxK)
        hipLaunchKernelGGL(k_bias_pixels<kBiasMaxK>, dim3(bx, m), dim3(kBlock), 0, st, geo, pose, centres, inv2w2,
                           beta, K, pred_biased, bias, grad, partial, bx);
    else
        return hipErrorInvalidValue;
    const int64_t nt = (int64_t)m * (K + 6);
    hipLaunchKernelGGL(k_bias_slices, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, (const float*)partial,
                       m, K, bx, terms);
    if (g_beta && s_n > 0 && K > 0)
        hipLaunchKernelGGL(k_bias_beta, dim3((unsigned)(((int64_t)s_n * K + 255) / 256)), dim3(256), 0, st,
                           (const float*)terms, subj, s_n, K, g_beta);
    if (g_pose)
        hipLaunchKernelGGL(k_bias_pose, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, (const float*)terms,
                           pose, m, K, g_pose);
    return hipGetLastError();
}

}  // namespace svr
