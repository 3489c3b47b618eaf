// AdamW over all parameter groups in one launch (App. A.1 optimiser),
// following torch.optim.AdamW's update order.
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kMaxSegs = 8;
struct AdamArgs {
    AdamSeg seg[kMaxSegs];
    int64_t start[kMaxSegs + 1];
    int n_segs;
    float beta2, omb1, omb2, eps, wd;  // omb = 1 - beta, formed in double on the host
    float bc1, bc2_sqrt;  // 1 - beta1^t, sqrt(1 - beta2^t)
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a, float* __restrict__ m, float* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.start[a.n_segs]) return;
    int s = 0;
    while (s + 1 < a.n_segs && i >= a.start[s + 1]) ++s;
    const AdamSeg& g = a.seg[s];
    const int64_t e = i - a.start[s];
    const float lr = (g.pose_layout && (e % 6) >= 3) ? g.lr_b : g.lr_a;
    const int64_t k = g.state_off + e;
    const float gr = g.g[e];
    float p = g.p[e] * (1.f - lr * a.wd);
    float mm = m[k], vv = v[k];
    mm = mm + a.omb1 * (gr - mm);
    vv = vv * a.beta2 + a.omb2 * gr * gr;
    const float denom = sqrtf(vv) / a.bc2_sqrt + a.eps;
    p = p - (lr / a.bc1) * (mm / denom);
    m[k] = mm;
    v[k] = vv;
    g.p[e] = p;
}

}  // namespace

hipError_t launch_adam(const AdamSeg* segs, int n_segs, float* m, float* v, double beta1, double beta2,
                       double eps, double wd, int64_t step, hipStream_t st) {
    if (n_segs > kMaxSegs) return hipErrorInvalidValue;
    AdamArgs a;
    a.n_segs = n_segs;
    a.start[0] = 0;
    for (int s = 0; s < n_segs; ++s) {
        a.seg[s] = segs[s];
        a.start[s + 1] = a.start[s] + segs[s].n;
    }
    for (int s = n_segs; s < kMaxSegs; ++s) a.start[s + 1] = a.start[n_segs];
    a.beta2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    a.wd = (float)wd;
    a.bc1 = (float)(1.0 - pow(beta1, (double)step));
    a.bc2_sqrt = (float)sqrt(1.0 - pow(beta2, (double)step));
    const int64_t n = a.start[n_segs];
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, m, v);
    return hipGetLastError();
}

}  // namespace svr
