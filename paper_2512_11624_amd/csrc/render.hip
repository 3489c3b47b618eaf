// Tile stages: per-tile instance ranges, the forward accumulation with the
// masked-MSE epilogue, and the adjoint.  gfx950, wave64, FP32.
//
// Forward (pixel per lane): a workgroup owns one T x T pixel tile of one
// slice.  Records of the tile are staged in LDS in batches; each wave owns a
// band of rows and skips records whose footprint rows miss its band.  The
// exponent of a record at tile-local pixel (X, Y) (relative to the tile
// centre) is the quadratic c0 + c1 X + c2 Y + c3 X^2 + c4 XY + c5 Y^2 whose
// coefficients are formed once per record at staging, so a pixel-record term
// costs 5 FMA, one exp2 and the window max(e - e_T, 0).  Every pixel sums its
// records in the sorted (deterministic) order.
//
// Adjoint (record per lane): the tile's upstream gradients are staged in LDS;
// each lane owns one instance and walks the pixels of its record's footprint
// box inside the tile, accumulating the seven moment sums it needs in
// registers (no cross-lane reduction), then adds them to the record's
// gradient with one atomic per component.
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kMaxBatch = 256;

__device__ inline int xcd_tile(int b, int n_tiles) {
    // consecutive tiles (which share records) go to the same XCD / L2
    const int per = (n_tiles + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, int64_t n, int2* __restrict__ ranges,
                              uint32_t n_tiles) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t k = keys[s];
    if (k >= n_tiles) return;
    if (s == 0 || keys[s - 1] != k) ranges[k].x = (int)s;
    if (s == n - 1 || keys[s + 1] != k) ranges[k].y = (int)(s + 1);
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_partial_sum(const float* __restrict__ x, int64_t n,
                                                      float* __restrict__ partial) {
    __shared__ float s[4];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc += x[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void k_final_sum(const float* __restrict__ partial, int n,
                                                    float* __restrict__ out) {
    __shared__ float s[4];
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = s[0] + s[1] + s[2] + s[3];
}

// One workgroup per slice: sum of the slice's tile partials.
__global__ __launch_bounds__(256) void k_slice_sse(const float* __restrict__ tile_sse,
                                                    const SliceGeo* __restrict__ geo,
                                                    float* __restrict__ slice_sse) {
    __shared__ float s[4];
    const SliceGeo& g = geo[blockIdx.x];
    const int nt = g.ntx * g.nty;
    float acc = 0.f;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) acc += tile_sse[g.tile_base + t];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) slice_sse[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ slice_sse, int m,
                                              const float* __restrict__ msum, float* __restrict__ loss) {
    __shared__ float s[4];
    float acc = 0.f;
    for (int i = threadIdx.x; i < m; i += blockDim.x) acc += slice_sse[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float ms = msum[0];
        loss[0] = ms > 0.f ? (s[0] + s[1] + s[2] + s[3]) / ms : 0.f;
    }
}

struct TileCoord {
    int slice, x0, y0, W, H;
    int64_t pix_off;
};

__device__ inline TileCoord tile_coord(const RenderArgs& a, int tile) {
    TileCoord c;
    c.slice = a.tile_slice[tile];
    const SliceGeo& g = a.geo[c.slice];
    const int local = tile - g.tile_base;
    const int ty = local / g.ntx, tx = local - ty * g.ntx;
    c.x0 = tx * a.tile;
    c.y0 = ty * a.tile;
    c.W = g.W;
    c.H = g.H;
    c.pix_off = g.pix_off;
    return c;
}

// Returns the next tile of this workgroup, or -1.
template <int NT>
__device__ inline int next_tile(const RenderArgs& a, int* work_counter, int& it, int* s_next) {
    if (!a.persistent) {
        if (it++ > 0) return -1;
        const int t = xcd_tile(blockIdx.x, a.n_tiles);
        return t < a.n_tiles ? t : -2;  // -2: idle block of the XCD remap
    }
    if (threadIdx.x == 0) *s_next = atomicAdd(work_counter, 1);
    __syncthreads();
    const int q = *s_next;
    __syncthreads();
    if (q >= a.n_tiles) return -1;
    return a.tile_order ? a.tile_order[q] : q;
}

template <int T, int PPT, bool kLoss, bool kCount>
__global__ __launch_bounds__(T * T / PPT) void k_forward(RenderArgs a, const float* __restrict__ target,
                                                         const float* __restrict__ mask,
                                                         const float* __restrict__ msum,
                                                         float* __restrict__ pred,
                                                         float* __restrict__ grad,
                                                         float* __restrict__ tile_sse,
                                                         unsigned long long* __restrict__ incut,
                                                         int* __restrict__ work_counter) {
    constexpr int NT = T * T / PPT;
    constexpr int NW = NT / 64;
    constexpr int ROWS = PPT * 64 / T;  // rows per wave band
    __shared__ float s_c[6][kMaxBatch];
    __shared__ float s_amp[kMaxBatch];
    __shared__ float s_ylo[kMaxBatch];
    __shared__ float s_yhi[kMaxBatch];
    __shared__ float s_red[NW > 0 ? NW : 1];
    __shared__ unsigned int s_cnt[NW > 0 ? NW : 1];
    __shared__ int s_next;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float hc = 0.5f * (float)(T - 1);
    const float band_lo = (float)(wv * ROWS) - 0.5f, band_hi = (float)(wv * ROWS + ROWS - 1) + 0.5f;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;  // KZ * T^2
    float X[PPT], Y[PPT];
    int lx[PPT], ly[PPT];
    for (int k = 0; k < PPT; ++k) {
        const int p = (wv * PPT + k) * 64 + lane;
        lx[k] = p % T;
        ly[k] = p / T;
        X[k] = (float)lx[k] - hc;
        Y[k] = (float)ly[k] - hc;
    }
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile == -1) break;
        if (tile == -2) break;
        const TileCoord tc = tile_coord(a, tile);
        const int2 rg = a.ranges[tile];
        float acc[PPT];
        for (int k = 0; k < PPT; ++k) acc[k] = 0.f;
        unsigned int cnt = 0;
        for (int b0 = rg.x; b0 < rg.y; b0 += a.batch) {
            const int nb = min(a.batch, rg.y - b0);
            __syncthreads();
            for (int q = tid; q < nb; q += NT) {
                const Record R = a.rec[a.inst_rec[b0 + q]];
                const float PX = R.r0.x - (float)tc.x0 - hc, PY = R.r0.y - (float)tc.y0 - hc;
                const float a00 = R.r1.x, a01 = R.r1.y, a11 = R.r1.z;
                s_c[0][q] = R.r0.z + PX * (a00 * PX + 2.f * a01 * PY) + a11 * PY * PY;
                s_c[1][q] = -2.f * (a00 * PX + a01 * PY);
                s_c[2][q] = -2.f * (a01 * PX + a11 * PY);
                s_c[3][q] = a00;
                s_c[4][q] = 2.f * a01;
                s_c[5][q] = a11;
                s_amp[q] = R.r0.w;
                // footprint row extent (tile-local rows)
                const float det = a00 * a11 - a01 * a01;
                const float hy = sqrtf(fmaxf((tau2k - R.r0.z) * a00 / det, 0.f)) + 1e-3f;
                const float cy = R.r0.y - (float)tc.y0;
                s_ylo[q] = cy - hy;
                s_yhi[q] = cy + hy;
            }
            __syncthreads();
            for (int q = 0; q < nb; ++q) {
                if (NW > 1 && (s_ylo[q] > band_hi || s_yhi[q] < band_lo)) continue;
                const float c0 = s_c[0][q], c1 = s_c[1][q], c2 = s_c[2][q];
                const float c3 = s_c[3][q], c4 = s_c[4][q], c5 = s_c[5][q], am = s_amp[q];
                for (int k = 0; k < PPT; ++k) {
                    float z = fmaf(c1, X[k], c0);
                    z = fmaf(c2, Y[k], z);
                    z = fmaf(c3, X[k] * X[k], z);
                    z = fmaf(c4, X[k] * Y[k], z);
                    z = fmaf(c5, Y[k] * Y[k], z);
                    const float e = __builtin_amdgcn_exp2f(z);
                    const float v = fmaxf(e - etau, 0.f);
                    acc[k] = fmaf(am, v, acc[k]);
                    if (kCount) cnt += (v > 0.f) ? 1u : 0u;
                }
            }
        }
        // epilogue
        float sq = 0.f;
        for (int k = 0; k < PPT; ++k) {
            const int px = tc.x0 + lx[k], py = tc.y0 + ly[k];
            if (px < tc.W && py < tc.H) {
                const int64_t pi = tc.pix_off + (int64_t)py * tc.W + px;
                pred[pi] = acc[k];
                if (kLoss) {
                    const float m = mask[pi];
                    const float r = acc[k] - target[pi];
                    sq = fmaf(m * r, r, sq);
                    if (grad) grad[pi] = 2.f * m * r * inv_msum;
                }
            }
        }
        if (kLoss || kCount) {
            for (int o = 32; o > 0; o >>= 1) {
                sq += __shfl_xor(sq, o, 64);
                if (kCount) cnt += __shfl_xor(cnt, o, 64);
            }
            if (lane == 0) {
                s_red[wv] = sq;
                s_cnt[wv] = cnt;
            }
            __syncthreads();
            if (tid == 0) {
                float t = 0.f;
                unsigned long long c = 0;
                for (int q = 0; q < NW; ++q) {
                    t += s_red[q];
                    c += s_cnt[q];
                }
                if (kLoss) tile_sse[tile] = t;
                if (kCount && c) atomicAdd(incut, c);
            }
        }
    }
}

template <int T, int PPT>
__global__ __launch_bounds__(T * T / PPT) void k_backward(RenderArgs a, const float* __restrict__ grad_pred,
                                                          const float* __restrict__ grad_scale,
                                                          RecGrad* __restrict__ rgrad,
                                                          int* __restrict__ work_counter) {
    constexpr int NT = T * T / PPT;
    constexpr int NW = NT / 64;
    __shared__ float s_g[T * T];
    __shared__ int s_next;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float scale = grad_scale ? grad_scale[0] : 1.f;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile == -1 || tile == -2) break;
        const TileCoord tc = tile_coord(a, tile);
        const int2 rg = a.ranges[tile];
        __syncthreads();
        for (int p = tid; p < T * T; p += NT) {
            const int px = tc.x0 + p % T, py = tc.y0 + p / T;
            float g = 0.f;
            if (px < tc.W && py < tc.H) g = grad_pred[tc.pix_off + (int64_t)py * tc.W + px] * scale;
            s_g[p] = g;
        }
        __syncthreads();
        const int n = rg.y - rg.x;
        for (int c0 = wv * 64; c0 < n; c0 += NW * 64) {
            const int s = c0 + lane;
            if (s >= n) continue;
            const uint32_t rid = a.inst_rec[rg.x + s];
            const Record R = a.rec[rid];
            const float pxl = R.r0.x - (float)tc.x0, pyl = R.r0.y - (float)tc.y0;
            const float bz = R.r0.z, am = R.r0.w;
            const float a00 = R.r1.x, a01 = R.r1.y, a11 = R.r1.z;
            const float det = a00 * a11 - a01 * a01;
            const float rk = tau2k - bz;  // KZ (T^2 - beta) <= 0
            const float hx = sqrtf(fmaxf(rk * a11 / det, 0.f)) + 1e-3f;
            const float hy = sqrtf(fmaxf(rk * a00 / det, 0.f)) + 1e-3f;
            const int x0 = max((int)ceilf(pxl - hx), 0), x1 = min((int)floorf(pxl + hx), T - 1);
            const int y0 = max((int)ceilf(pyl - hy), 0), y1 = min((int)floorf(pyl + hy), T - 1);
            float S0 = 0.f, Sx = 0.f, Sy = 0.f, Sxx = 0.f, Sxy = 0.f, Syy = 0.f, Sa = 0.f;
            if (x0 <= x1 && y0 <= y1) {
                const float a01x2 = 2.f * a01;
                for (int y = y0; y <= y1; ++y) {
                    const float dy = (float)y - pyl;
                    const float zy = fmaf(a11 * dy, dy, bz);
                    const float bx = a01x2 * dy;
                    for (int x = x0; x <= x1; ++x) {
                        const float dx = (float)x - pxl;
                        const float z = fmaf(dx, fmaf(a00, dx, bx), zy);
                        const float e = __builtin_amdgcn_exp2f(z);
                        const float g = s_g[y * T + x];
                        const float v = e - etau;
                        Sa = fmaf(g, fmaxf(v, 0.f), Sa);
                        const float t = (v > 0.f) ? g * e : 0.f;
                        const float tx = t * dx;
                        S0 += t;
                        Sx += tx;
                        Sy = fmaf(t, dy, Sy);
                        Sxx = fmaf(tx, dx, Sxx);
                        Sxy = fmaf(tx, dy, Sxy);
                        Syy = fmaf(t * dy, dy, Syy);
                    }
                }
            }
            // dz/d(stored) with t = g e, times amp * ln 2
            const float k2 = am * SVR_LN2;
            const float dbz = k2 * S0;
            const float dpx = -2.f * k2 * (a00 * Sx + a01 * Sy);
            const float dpy = -2.f * k2 * (a01 * Sx + a11 * Sy);
            const float da00 = k2 * Sxx, da01 = 2.f * k2 * Sxy, da11 = k2 * Syy;
            float* dst = rgrad[rid].v;
            if (Sa != 0.f) unsafeAtomicAdd(dst + 0, Sa);
            if (S0 != 0.f) {
                unsafeAtomicAdd(dst + 1, dbz);
                unsafeAtomicAdd(dst + 2, dpx);
                unsafeAtomicAdd(dst + 3, dpy);
                unsafeAtomicAdd(dst + 4, da00);
                unsafeAtomicAdd(dst + 5, da01);
                unsafeAtomicAdd(dst + 6, da11);
            }
        }
    }
}

template <int T, int PPT>
hipError_t fwd_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                        float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                        int* work_counter, int grid, hipStream_t st) {
    constexpr int NT = T * T / PPT;
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    if (loss && count)
        hipLaunchKernelGGL((k_forward<T, PPT, true, true>), dim3(grid), dim3(NT), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else if (loss)
        hipLaunchKernelGGL((k_forward<T, PPT, true, false>), dim3(grid), dim3(NT), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else if (count)
        hipLaunchKernelGGL((k_forward<T, PPT, false, true>), dim3(grid), dim3(NT), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else
        hipLaunchKernelGGL((k_forward<T, PPT, false, false>), dim3(grid), dim3(NT), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    return hipGetLastError();
}

int grid_for(const RenderArgs& a, int threads) {
    if (a.persistent) {
        const int cus = a.n_cu > 0 ? a.n_cu : 256;
        const int per_cu = threads >= 256 ? 8 : 16;
        const int g = cus * per_cu;
        return g < a.n_tiles ? g : (a.n_tiles > 0 ? a.n_tiles : 1);
    }
    return ((a.n_tiles + 7) >> 3) << 3;
}

__global__ void k_tile_cost_keys(const int2* __restrict__ ranges, int32_t n, uint32_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int2 r = ranges[t];
    const int c = min(r.y - r.x, 0xffff);
    keys[t] = (uint32_t)(0xffff - c);  // ascending key = descending cost
    vals[t] = (uint32_t)t;
}

}  // namespace

hipError_t launch_tile_cost_keys(const int2* ranges, int32_t n_tiles, uint32_t* keys, uint32_t* vals,
                                 hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_cost_keys, dim3((n_tiles + 255) / 256), dim3(256), 0, st, ranges, n_tiles, keys, vals);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* keys, int64_t n, int2* ranges, int32_t n_tiles,
                              hipStream_t st) {
    hipError_t e = launch_fill_zero(ranges, sizeof(int2) * (size_t)n_tiles, st);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, n, ranges,
                       (uint32_t)n_tiles);
    return hipGetLastError();
}

hipError_t launch_mask_sum(const float* mask, int64_t n, float* partial, float* out, hipStream_t st) {
    const int nb = 1024;
    hipLaunchKernelGGL(k_partial_sum, dim3(nb), dim3(256), 0, st, mask, n, partial);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, (const float*)partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_forward(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                          float* pred, float* grad_pred, float* tile_sse, unsigned long long* incut,
                          int* work_counter, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (a.persistent) {
        hipError_t e = launch_fill_zero(work_counter, sizeof(int), st);
        if (e != hipSuccess) return e;
    }
    switch (a.tile) {
        case 8: return fwd_dispatch<8, 1>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 64), st);
        case 16: return fwd_dispatch<16, 1>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 256), st);
        case 32: return fwd_dispatch<32, 4>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 256), st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_loss_finalize(const float* tile_sse, const SliceGeo* geo, int32_t m, const float* msum,
                                float* slice_sse, float* loss, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_sse, dim3(m), dim3(256), 0, st, tile_sse, geo, slice_sse);
    if (loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, (const float*)slice_sse, m, msum, loss);
    return hipGetLastError();
}

hipError_t launch_backward(const RenderArgs& a, const float* grad_pred, const float* grad_scale,
                           RecGrad* rgrad, int* work_counter, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (a.persistent) {
        hipError_t e = launch_fill_zero(work_counter, sizeof(int), st);
        if (e != hipSuccess) return e;
    }
    switch (a.tile) {
        case 8:
            hipLaunchKernelGGL((k_backward<8, 1>), dim3(grid_for(a, 64)), dim3(64), 0, st, a, grad_pred, grad_scale, rgrad, work_counter);
            break;
        case 16:
            hipLaunchKernelGGL((k_backward<16, 1>), dim3(grid_for(a, 256)), dim3(256), 0, st, a, grad_pred, grad_scale, rgrad, work_counter);
            break;
        case 32:
            hipLaunchKernelGGL((k_backward<32, 4>), dim3(grid_for(a, 256)), dim3(256), 0, st, a, grad_pred, grad_scale, rgrad, work_counter);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace svr
