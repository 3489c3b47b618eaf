// AdamW over all parameter groups in one launch (App. A.1 optimiser),
// following torch.optim.AdamW's update order.
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kMaxSegs = 8;
struct AdamArgs {
    AdamSeg seg[kMaxSegs];
    int64_t qstart[kMaxSegs + 1];  // first quad (four elements) of each segment
    int n_segs;
    float beta2, omb1, omb2, eps, wd;  // omb = 1 - beta, formed in double on the host
    float bc1, bc2_sqrt;  // 1 - beta1^t, sqrt(1 - beta2^t)
};

__device__ inline void adam_one(const AdamArgs& a, const AdamSeg& g, int64_t e, float& p, float gr, float& mm,
                                float& vv) {
    const float lr = (g.pose_layout && (e % 6) >= 3) ? g.lr_b : g.lr_a;
    p = p * (1.f - lr * a.wd);
    mm = mm + a.omb1 * (gr - mm);
    vv = vv * a.beta2 + a.omb2 * gr * gr;
    const float denom = sqrtf(vv) / a.bc2_sqrt + a.eps;
    p = p - (lr / a.bc1) * (mm / denom);
}

// Four consecutive elements of one segment per thread (segment s owns
// quads qstart[s] .. qstart[s + 1] - 1): 16-byte accesses when the four
// arrays are aligned there, element by element otherwise.  The arithmetic is
// per element, so the result does not depend on the grouping.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a, float* __restrict__ m, float* __restrict__ v) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.qstart[a.n_segs]) return;
    int s = 0;
    while (s + 1 < a.n_segs && q >= a.qstart[s + 1]) ++s;
    const AdamSeg& g = a.seg[s];
    const int64_t e0 = 4 * (q - a.qstart[s]);
    const int64_t k0 = g.state_off + e0;
    const bool full = e0 + 3 < g.n;
    const bool aligned = ((reinterpret_cast<uintptr_t>(g.p + e0) | reinterpret_cast<uintptr_t>(g.g + e0) |
                           reinterpret_cast<uintptr_t>(m + k0) | reinterpret_cast<uintptr_t>(v + k0)) & 15) == 0;
    if (full && aligned) {
        float4 p4 = *reinterpret_cast<const float4*>(g.p + e0);
        const float4 g4 = *reinterpret_cast<const float4*>(g.g + e0);
        float4 m4 = *reinterpret_cast<const float4*>(m + k0);
        float4 v4 = *reinterpret_cast<const float4*>(v + k0);
        adam_one(a, g, e0, p4.x, g4.x, m4.x, v4.x);
        adam_one(a, g, e0 + 1, p4.y, g4.y, m4.y, v4.y);
        adam_one(a, g, e0 + 2, p4.z, g4.z, m4.z, v4.z);
        adam_one(a, g, e0 + 3, p4.w, g4.w, m4.w, v4.w);
        *reinterpret_cast<float4*>(m + k0) = m4;
        *reinterpret_cast<float4*>(v + k0) = v4;
        *reinterpret_cast<float4*>(g.p + e0) = p4;
        return;
    }
    for (int j = 0; j < 4; ++j) {
        const int64_t e = e0 + j;
        if (e >= g.n) break;
        float p = g.p[e], mm = m[k0 + j], vv = v[k0 + j];
        adam_one(a, g, e, p, g.g[e], mm, vv);
        m[k0 + j] = mm;
        v[k0 + j] = vv;
        g.p[e] = p;
    }
}

}  // namespace

hipError_t launch_adam(const AdamSeg* segs, int n_segs, float* m, float* v, double beta1, double beta2,
                       double eps, double wd, int64_t step, hipStream_t st) {
    if (n_segs > kMaxSegs) return hipErrorInvalidValue;
    AdamArgs a;
    a.n_segs = n_segs;
    a.qstart[0] = 0;
    for (int s = 0; s < n_segs; ++s) {
        a.seg[s] = segs[s];
        a.qstart[s + 1] = a.qstart[s] + (segs[s].n + 3) / 4;
    }
    for (int s = n_segs; s < kMaxSegs; ++s) a.qstart[s + 1] = a.qstart[n_segs];
    a.beta2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    a.wd = (float)wd;
    a.bc1 = (float)(1.0 - pow(beta1, (double)step));
    a.bc2_sqrt = (float)sqrt(1.0 - pow(beta2, (double)step));
    const int64_t nq = a.qstart[n_segs];
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, a, m, v);
    return hipGetLastError();
}

}  // namespace svr
