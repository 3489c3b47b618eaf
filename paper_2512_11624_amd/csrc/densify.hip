// Adaptive densification of the Gaussian mixture (the coarse-to-fine
// optimisation the paper leaves to future work, Sec. 4, after the clone/split
// scheme of 3D Gaussian Splatting).
//
// Statistic: every step adds ||dL/dmu_j|| to A_j and 1 to n_j when the mean
// gradient is not zero.  Decision (FP32, one rounding in the bound):
// prune when |c_j| < prune_amp (0 outputs), densify when n_j > 0 and
// A_j > fl(grad_threshold * n_j) (2 outputs), else keep (1 output).  A
// densified Gaussian splits when its largest log-scale exceeds
// log_scale_threshold and clones otherwise.  Children sit at mu -+ o s_a e on
// the principal axis e (column a of R(q) for the largest scale s_a, the first
// on ties) with o the split or clone offset; a split also shrinks s_a by
// sqrt(1 - a^2) and scales the amplitude by 1 / (2 sqrt(1 - a^2)), which keeps
// the parent's integral and first two moments; a clone halves the amplitude.
//
// Passes: decide (one thread per Gaussian) -> exclusive scan of the output
// counts -> per-subject output offsets (read back: the caller sizes the next
// step by them) -> emit (one thread per parent writes its 0, 1 or 2 outputs
// at its scanned position, so the outputs keep subject and parent order).
// Every pass is a streaming read/write of the per-Gaussian arrays; none needs
// LDS.
#include "svr_internal.h"

namespace svr {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_dens_accum(const float* __restrict__ g_mean, float* __restrict__ acc,
                                                       int32_t* __restrict__ cnt, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const float gx = g_mean[3 * j], gy = g_mean[3 * j + 1], gz = g_mean[3 * j + 2];
    acc[j] += sqrtf(gx * gx + gy * gy + gz * gz);
    cnt[j] += (gx != 0.f || gy != 0.f || gz != 0.f) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_dens_decide(const float* __restrict__ acc, const int32_t* __restrict__ cnt,
                                                        const float* __restrict__ amp, int64_t n, float grad_thr,
                                                        float prune_amp, int32_t* __restrict__ n_out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int32_t c = cnt[j];
    const bool dens = c > 0 && acc[j] > __fmul_rn(grad_thr, (float)c);
    const bool prune = fabsf(amp[j]) < prune_amp;
    n_out[j] = prune ? 0 : (dens ? 2 : 1);
}

// new_off[s] = first output of subject s (s = 0..S; new_off[S] = total)
__global__ void k_dens_offsets(const int32_t* __restrict__ pos, const SubjectInfo* __restrict__ subj, int32_t S,
                               int64_t n, const long long* __restrict__ total, int64_t* __restrict__ new_off) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S) return;
    const int64_t g = s < S ? subj[s].g_begin : n;
    new_off[s] = g < n ? (int64_t)pos[g] : (int64_t)total[0];
}

__global__ __launch_bounds__(kBlock) void k_dens_emit(DensifyArgs a) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    const int32_t no = a.n_out[j];
    if (no == 0) return;
    const int64_t k = a.pos[j];
    float mu[3], ls[3], q[4];
    for (int d = 0; d < 3; ++d) mu[d] = a.mean[3 * j + d];
    for (int d = 0; d < 3; ++d) ls[d] = a.log_scale[3 * j + d];
    for (int d = 0; d < 4; ++d) q[d] = a.quat[4 * j + d];
    const float c = a.amp[j];
    const int64_t N = a.n, K = a.n_new;
    if (no == 1) {
        for (int d = 0; d < 3; ++d) a.o_mean[3 * k + d] = mu[d];
        for (int d = 0; d < 3; ++d) a.o_log_scale[3 * k + d] = ls[d];
        for (int d = 0; d < 4; ++d) a.o_quat[4 * k + d] = q[d];
        a.o_amp[k] = c;
        if (a.src) a.src[k] = (int32_t)j;
        for (int t = 0; t < 2; ++t) {
            const float* mi = t ? a.m2_in : a.m1_in;
            float* mo = t ? a.m2_out : a.m1_out;
            if (!mi) continue;
            for (int d = 0; d < 3; ++d) mo[3 * k + d] = mi[3 * j + d];
            for (int d = 0; d < 3; ++d) mo[3 * K + 3 * k + d] = mi[3 * N + 3 * j + d];
            for (int d = 0; d < 4; ++d) mo[6 * K + 4 * k + d] = mi[6 * N + 4 * j + d];
            mo[10 * K + k] = mi[10 * N + j];
        }
        return;
    }
    // principal axis: the first largest log-scale
    int ax = 0;
    if (ls[1] > ls[ax]) ax = 1;
    if (ls[2] > ls[ax]) ax = 2;
    const float inv = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
    float e[3];
    if (ax == 0) {
        e[0] = 1.f - 2.f * (y * y + z * z); e[1] = 2.f * (x * y + w * z); e[2] = 2.f * (x * z - w * y);
    } else if (ax == 1) {
        e[0] = 2.f * (x * y - w * z); e[1] = 1.f - 2.f * (x * x + z * z); e[2] = 2.f * (y * z + w * x);
    } else {
        e[0] = 2.f * (x * z + w * y); e[1] = 2.f * (y * z - w * x); e[2] = 1.f - 2.f * (x * x + y * y);
    }
    const bool split = ls[ax] > a.log_scale_thr;
    const float o = (split ? a.split_offset : a.clone_offset) * expf(ls[ax]);
    float lc[3] = {ls[0], ls[1], ls[2]};
    if (split) lc[ax] += a.split_dlog;
    const float cc = c * (split ? a.split_amp : 0.5f);
    for (int h = 0; h < 2; ++h) {
        const int64_t kk = k + h;
        const float sg = h ? 1.f : -1.f;
        for (int d = 0; d < 3; ++d) a.o_mean[3 * kk + d] = fmaf(sg * o, e[d], mu[d]);
        for (int d = 0; d < 3; ++d) a.o_log_scale[3 * kk + d] = lc[d];
        for (int d = 0; d < 4; ++d) a.o_quat[4 * kk + d] = q[d];
        a.o_amp[kk] = cc;
        if (a.src) a.src[kk] = (int32_t)(-(j + 1));
        for (int t = 0; t < 2; ++t) {
            float* mo = t ? a.m2_out : a.m1_out;
            if (!mo) continue;
            for (int d = 0; d < 3; ++d) mo[3 * kk + d] = 0.f;
            for (int d = 0; d < 3; ++d) mo[3 * K + 3 * kk + d] = 0.f;
            for (int d = 0; d < 4; ++d) mo[6 * K + 4 * kk + d] = 0.f;
            mo[10 * K + kk] = 0.f;
        }
    }
}

}  // namespace

hipError_t launch_densify_accumulate(const float* g_mean, float* acc, int32_t* cnt, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dens_accum, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, g_mean, acc,
                       cnt, n);
    return hipGetLastError();
}

hipError_t launch_densify_plan(const float* acc, const int32_t* cnt, const float* amp, int64_t n, float grad_thr,
                               float prune_amp, const SubjectInfo* subj, int32_t S, int32_t* n_out, int32_t* pos,
                               long long* total, void* scan_tmp, int64_t* new_off, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_dens_decide, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, acc, cnt,
                           amp, n, grad_thr, prune_amp, n_out);
    hipError_t e = launch_scan_int(n_out, pos, n, total, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dens_offsets, dim3((unsigned)((S + 1 + 255) / 256)), dim3(256), 0, st, (const int32_t*)pos,
                       subj, S, n, (const long long*)total, new_off);
    return hipGetLastError();
}

hipError_t launch_densify_emit(const DensifyArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dens_emit, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace svr
