// Content-adaptive initialisation of the Gaussian means (Sec. 2.5, Eq. 6).
//
// The means are drawn from a density over the slices' pixels proportional to
// (1 - lambda) ||grad I|| / max ||grad I|| + lambda (masked pixels only).
// The weight of a pixel is quantised to an integer (2^20 per unit of the
// density) in FP64 with every operation rounded once, so that the discrete
// draw is an exact integer decision that does not depend on summation order:
//   1. k_init_grad     ||grad I|| per pixel (FP64), and its maximum over each
//                      subject's masked pixels (integer atomic max on the bits);
//   2. k_init_scan1    quantised weights, inclusive scan within blocks of
//                      4096 pixels, block totals;
//   3. k_init_scan2    exclusive scan of the block totals (one workgroup);
//   4. k_init_bases    each subject's base and total weight;
//   5. k_init_scan3    final cumulative weights, restarting at each subject;
//   6. k_init_sample   per Gaussian: inverse-CDF draw of a pixel of its
//                      subject, then the world position of a uniform point in
//                      that pixel's footprint and slab.
// All int64 sums are exact; the cumulative weights are the same on any grid.
#include <algorithm>

#include "svr_internal.h"

#pragma clang fp contract(off)

namespace svr {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;   // pixels per scan block
constexpr double kQuant = 1048576.0;     // 2^20

__device__ inline int64_t subject_of_pixel(const int64_t* __restrict__ sub_pix, int s_n, int64_t p) {
    int lo = 0, hi = s_n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sub_pix[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ||grad I|| per mm of pixel (r, k) of slice i: central differences inside,
// one-sided on the border, 0 along an axis of length 1.
__global__ __launch_bounds__(kBlock) void k_init_grad(const SliceGeo* __restrict__ geo,
                                                      const InitSlice* __restrict__ tab, int32_t m,
                                                      const float* __restrict__ image,
                                                      const float* __restrict__ mask, double* __restrict__ g,
                                                      unsigned long long* __restrict__ gmax_bits) {
    __shared__ double s_max[kBlock / 64];
    for (int32_t i = blockIdx.y; i < m; i += gridDim.y) {
        const SliceGeo& sg = geo[i];
        const InitSlice& it = tab[i];
        const int H = sg.H, W = sg.W;
        const int64_t n = (int64_t)H * W;
        const float* img = image + sg.pix_off;
        double best = 0.0;
        for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBlock) {
            const int r = (int)(q / W), k = (int)(q - (int64_t)r * W);
            double gx = 0.0, gy = 0.0;
            if (W > 1) {
                if (k == 0) gx = ((double)img[q + 1] - (double)img[q]) * it.inv1_x;
                else if (k == W - 1) gx = ((double)img[q] - (double)img[q - 1]) * it.inv1_x;
                else gx = ((double)img[q + 1] - (double)img[q - 1]) * it.inv2_x;
            }
            if (H > 1) {
                if (r == 0) gy = ((double)img[q + W] - (double)img[q]) * it.inv1_y;
                else if (r == H - 1) gy = ((double)img[q] - (double)img[q - W]) * it.inv1_y;
                else gy = ((double)img[q + W] - (double)img[q - W]) * it.inv2_y;
            }
            const double gm = __builtin_sqrt(gx * gx + gy * gy);
            g[sg.pix_off + q] = gm;
            if (!mask || mask[sg.pix_off + q] > 0.f) best = fmax(best, gm);
        }
        for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
        if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double b = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
            // nonnegative doubles order like their bit patterns
            if (b > 0.0) atomicMax(gmax_bits + sg.subject, (unsigned long long)__double_as_longlong(b));
        }
        __syncthreads();
    }
}

__device__ inline int64_t quantised_weight(double gm, double gmax, double lam, bool on) {
    if (!on) return 0;
    const double p = gmax > 0.0 ? (1.0 - lam) * (gm / gmax) + lam : lam;
    return (int64_t)floor(p * kQuant);
}

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* s_wave, int64_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) before += s_wave[w];
        total += s_wave[w];
    }
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_init_scan1(const double* __restrict__ g, const float* __restrict__ mask,
                                                       int64_t P, const int64_t* __restrict__ sub_pix, int32_t s_n,
                                                       const unsigned long long* __restrict__ gmax_bits, double lam,
                                                       int64_t* __restrict__ cdf, int64_t* __restrict__ bsum) {
    __shared__ int64_t s_wave[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t w[kItems];
    int64_t run = 0;
    int64_t s = base < P ? subject_of_pixel(sub_pix, s_n, base) : 0;
    for (int k = 0; k < kItems; ++k) {
        const int64_t p = base + k;
        int64_t wk = 0;
        if (p < P) {
            while (s + 1 < s_n && sub_pix[s + 1] <= p) ++s;
            const double gmax = __longlong_as_double((long long)gmax_bits[s]);
            wk = quantised_weight(g[p], gmax, lam, !mask || mask[p] > 0.f);
        }
        run += wk;
        w[k] = run;
    }
    int64_t total;
    const int64_t before = block_exclusive_scan(run, s_wave, total);
    for (int k = 0; k < kItems; ++k) {
        const int64_t p = base + k;
        if (p < P) cdf[p] = before + w[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the block totals in place (one workgroup).
__global__ __launch_bounds__(kBlock) void k_init_scan2(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t s_wave[kBlock / 64];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? bsum[b] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, s_wave, total);
        if (b < nb) bsum[b] = carry + ex;
        carry += total;
    }
}

__device__ inline int64_t global_cdf(const int64_t* cdf, const int64_t* boff, int64_t p) {
    return boff[p / kTile] + cdf[p];
}

// Subject s: base = cumulative weight before its first pixel, total = its own.
__global__ void k_init_bases(const int64_t* __restrict__ cdf, const int64_t* __restrict__ boff,
                             const int64_t* __restrict__ sub_pix, int32_t s_n, int64_t* __restrict__ base,
                             int64_t* __restrict__ total) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= s_n) return;
    const int64_t a = sub_pix[s], b = sub_pix[s + 1];
    const int64_t lo = a > 0 ? global_cdf(cdf, boff, a - 1) : 0;
    base[s] = lo;
    total[s] = b > a ? global_cdf(cdf, boff, b - 1) - lo : 0;
}

__global__ __launch_bounds__(kBlock) void k_init_scan3(int64_t* __restrict__ cdf, const int64_t* __restrict__ boff,
                                                       int64_t P, const int64_t* __restrict__ sub_pix, int32_t s_n,
                                                       const int64_t* __restrict__ base) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    cdf[p] = global_cdf(cdf, boff, p) - base[subject_of_pixel(sub_pix, s_n, p)];
}

__global__ __launch_bounds__(kBlock) void k_init_sample(
        const SliceGeo* __restrict__ geo, const SlicePose* __restrict__ pose, const InitSlice* __restrict__ tab,
        const SubjectInfo* __restrict__ subj, int32_t s_n, const int64_t* __restrict__ sub_pix,
        const int64_t* __restrict__ cdf, const int64_t* __restrict__ total, const float* __restrict__ image,
        const float4* __restrict__ u, int64_t N, float* __restrict__ mean, int64_t* __restrict__ pixel,
        float* __restrict__ value) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= N) return;
    int s = 0;
    {
        int lo = 0, hi = s_n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (subj[mid].g_begin <= j) lo = mid; else hi = mid - 1;
        }
        s = lo;
    }
    const float4 uj = u[j];
    const int64_t W = total[s];
    int64_t t = (int64_t)floor((double)uj.x * (double)W);
    t = t < 0 ? 0 : (t > W - 1 ? W - 1 : t);
    // first pixel of the subject whose cumulative weight exceeds t
    int64_t lo = sub_pix[s], hi = sub_pix[s + 1] - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    const int64_t p = lo;
    int a = subj[s].s_begin, b = subj[s].s_end - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (geo[mid].pix_off <= p) a = mid; else b = mid - 1;
    }
    const SliceGeo& sg = geo[a];
    const SlicePose& sp = pose[a];
    const int64_t loc = p - sg.pix_off;
    const int r = (int)(loc / sg.W), k = (int)(loc - (int64_t)r * sg.W);
    const float x = ((float)k - 0.5f * (float)(sg.W - 1) + (uj.y - 0.5f)) * sg.dx;
    const float y = ((float)r - 0.5f * (float)(sg.H - 1) + (uj.z - 0.5f)) * sg.dy;
    const float z = (uj.w - 0.5f) * tab[a].thick;
    for (int c = 0; c < 3; ++c)
        mean[3 * j + c] = fmaf(sp.R[3 * c], x, fmaf(sp.R[3 * c + 1], y, fmaf(sp.R[3 * c + 2], z, sp.t[c])));
    if (pixel) pixel[j] = p;
    if (value) value[j] = image[p];
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

int64_t init_scan_blocks(int64_t P) { return (P + kTile - 1) / kTile; }

hipError_t launch_init_cdf(const SliceGeo* geo, const InitSlice* tab, int32_t m, int32_t max_hw,
                           const int64_t* sub_pix, int32_t s_n, int64_t P, const float* image, const float* mask,
                           float lambda, double* g, unsigned long long* gmax_bits, int64_t* cdf, int64_t* bsum,
                           int64_t* base, int64_t* total, hipStream_t st) {
    if (P <= 0 || m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((s_n + 255) / 256), dim3(256), 0, st, gmax_bits, s_n);
    const int gx = (int)std::min<int64_t>((max_hw + kBlock - 1) / kBlock, 1024);
    const int gy = std::min(m, 65535);
    hipLaunchKernelGGL(k_init_grad, dim3(gx, gy), dim3(kBlock), 0, st, geo, tab, m, image, mask, g, gmax_bits);
    const int64_t nb = init_scan_blocks(P);
    hipLaunchKernelGGL(k_init_scan1, dim3((unsigned)nb), dim3(kBlock), 0, st, (const double*)g, mask, P, sub_pix,
                       s_n, (const unsigned long long*)gmax_bits, (double)lambda, cdf, bsum);
    hipLaunchKernelGGL(k_init_scan2, dim3(1), dim3(kBlock), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_init_bases, dim3((s_n + 63) / 64), dim3(64), 0, st, (const int64_t*)cdf,
                       (const int64_t*)bsum, sub_pix, s_n, base, total);
    hipLaunchKernelGGL(k_init_scan3, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, cdf,
                       (const int64_t*)bsum, P, sub_pix, s_n, (const int64_t*)base);
    return hipGetLastError();
}

hipError_t launch_init_sample(const SliceGeo* geo, const SlicePose* pose, const InitSlice* tab,
                              const SubjectInfo* subj, int32_t s_n, const int64_t* sub_pix, const int64_t* cdf,
                              const int64_t* total, const float* image, const float* u, int64_t N, float* mean,
                              int64_t* pixel, float* value, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_sample, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, geo, pose,
                       tab, subj, s_n, sub_pix, cdf, total, image, (const float4*)u, N, mean, pixel, value);
    return hipGetLastError();
}

}  // namespace svr
