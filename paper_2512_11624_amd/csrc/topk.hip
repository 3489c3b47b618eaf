// Normalised Top-K forward model of Eqs. 2 and 5 (Sec. 2.2-2.5) and its
// adjoint.
//
// For pixel p of slice i at x = R_i u_p + t_i:
//   y_p = sigma_i * N_p / (D_p + delta),
//   N_p = sum_{j in S^K(x)} c_j e_j,  D_p = sum_{j in S^K(x)} e_j,
//   e_j = exp(-1/2 v^T Sigma_obs^-1 v), v = x - mu_j,
//   Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T,
// where S^K(x) are the K means of the slice's subject nearest to x (L2).
//
// Neighbour search (refreshed by the caller every few iterations, as the
// paper refreshes its index every 50 epochs):
//   k_bbox / host      per-subject bounding box and a uniform cell grid;
//   k_cell_keys, sort  Gaussians sorted by cell (stable, so by id within a
//                      cell), k_cell_ranges gives each cell's range;
//   k_knn              one wave per 8x8 pixel tile: the means inside
//                      the slab box that holds the radius-rho ball of every
//                      pixel of the tile are compacted into LDS in cell
//                      order; each lane (pixel) then selects its K nearest
//                      by two histogram passes over squared distance and an
//                      exact pick inside the boundary bin.  If some pixel
//                      has fewer than K means within rho, rho grows by 1.3;
//                      if the means within reach exceed LDS, the tile is
//                      split into 4x4, 2x2 and single-pixel sub-tiles, and a
//                      single pixel streams its candidates through LDS.
//   inverse lists      (Gaussian, pixel) pairs sorted by Gaussian, so that
//                      the adjoint gathers per Gaussian without atomics.
// Forward: one thread per pixel over its K neighbours.  Adjoint: a pixel
// pass for the slice pose and intensity scalar (per-slice partial sums, no
// atomics) and a Gaussian pass (one wave per Gaussian over its pixels).
#include <string.h>

#include <algorithm>

#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kBlock = 256;
constexpr int kTileSide = 16;
constexpr int kKnnSide = 8;      // neighbour search: one wave per 8x8 pixel tile
constexpr int kKnnThreads = kKnnSide * kKnnSide;
constexpr int kCandCap = 1024;   // means staged in LDS per (sub-)tile
constexpr int kBins = 64;
constexpr int kMaxTries = 20;

__device__ inline uint32_t float_order(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float order_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// --------------------------------------------------------------------------
// activation and per-slice constants
// --------------------------------------------------------------------------
// out[s] for Gaussian perm[s] (perm NULL: identity); the neighbour grid's
// cell order keeps spatial neighbours close in memory.
__global__ void k_topk_activate(const float* __restrict__ mean, const float* __restrict__ log_scale,
                                const float* __restrict__ quat, const float* __restrict__ amp, int64_t n,
                                const uint32_t* __restrict__ perm, TopkGauss* __restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t j = perm ? (int64_t)perm[s] : s;
    float qw = quat[4 * j], qx = quat[4 * j + 1], qy = quat[4 * j + 2], qz = quat[4 * j + 3];
    const float inv = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    float s2[3];
    for (int k = 0; k < 3; ++k) s2[k] = expf(2.f * log_scale[3 * j + k]);
    float S[6];  // 00 01 02 11 12 22
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
        float acc = 0.f;
        for (int k = 0; k < 3; ++k) acc = fmaf(R[3 * ia[e] + k] * s2[k], R[3 * ib[e] + k], acc);
        S[e] = acc;
    }
    TopkGauss g;
    g.a = make_float4(mean[3 * j], mean[3 * j + 1], mean[3 * j + 2], amp[j]);
    g.b = make_float4(S[0], S[1], S[2], S[3]);
    g.c = make_float4(S[4], S[5], 0.f, 0.f);
    out[s] = g;
}

__global__ void k_topk_slices(const SlicePose* __restrict__ pose, const SliceGeo* __restrict__ geo,
                              const float* __restrict__ sigma, int32_t m, TopkSlice* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const SlicePose& sp = pose[i];
    TopkSlice o;
    for (int k = 0; k < 9; ++k) o.R[k] = sp.R[k];
    for (int k = 0; k < 3; ++k) o.t[k] = sp.t[k];
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
        float acc = 0.f;
        for (int k = 0; k < 3; ++k) acc = fmaf(sp.R[3 * ia[e] + k] * geo[i].sig2[k], sp.R[3 * ib[e] + k], acc);
        o.P[e] = acc;
    }
    o.sigma = sigma ? sigma[i] : 1.f;
    o.pad[0] = o.pad[1] = o.pad[2] = 0.f;
    out[i] = o;
}

// e = exp(-1/2 v^T S^-1 v) and w = S^-1 v for a symmetric positive definite S.
__device__ inline float pair_eval(const float S[6], float vx, float vy, float vz, float& wx, float& wy,
                                  float& wz) {
    const float c00 = S[3] * S[5] - S[4] * S[4];
    const float c01 = S[2] * S[4] - S[1] * S[5];
    const float c02 = S[1] * S[4] - S[2] * S[3];
    const float c11 = S[0] * S[5] - S[2] * S[2];
    const float c12 = S[1] * S[2] - S[0] * S[4];
    const float c22 = S[0] * S[3] - S[1] * S[1];
    const float inv = 1.f / (S[0] * c00 + S[1] * c01 + S[2] * c02);
    wx = (c00 * vx + c01 * vy + c02 * vz) * inv;
    wy = (c01 * vx + c11 * vy + c12 * vz) * inv;
    wz = (c02 * vx + c12 * vy + c22 * vz) * inv;
    const float q = vx * wx + vy * wy + vz * wz;
    return exp2f(SVR_KZ * q);
}

__device__ inline float dist2(float px, float py, float pz, const float4& m) {
    const float dx = px - m.x, dy = py - m.y, dz = pz - m.z;
    return dx * dx + dy * dy + dz * dz;
}

__device__ inline void pixel_world(const SliceGeo& sg, const TopkSlice& ts, int r, int k, float& x, float& y,
                                   float& z, float& ux, float& uy) {
    ux = ((float)k - 0.5f * (float)(sg.W - 1)) * sg.dx;
    uy = ((float)r - 0.5f * (float)(sg.H - 1)) * sg.dy;
    x = fmaf(ts.R[0], ux, fmaf(ts.R[1], uy, ts.t[0]));
    y = fmaf(ts.R[3], ux, fmaf(ts.R[4], uy, ts.t[1]));
    z = fmaf(ts.R[6], ux, fmaf(ts.R[7], uy, ts.t[2]));
}

// --------------------------------------------------------------------------
// cell grid
// --------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// bb [s * 6 + (0..2 min, 3..5 max)] as order-preserving keys
__global__ void k_bbox(const float* __restrict__ mean, const GaussBlock* __restrict__ blocks, int32_t nb,
                       uint32_t* __restrict__ bb) {
    if ((int)blockIdx.x >= nb) return;
    const GaussBlock gb = blocks[blockIdx.x];
    const int64_t j = gb.g_begin + threadIdx.x;
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    if (j < gb.g_end)
        for (int k = 0; k < 3; ++k) lo[k] = hi[k] = float_order(mean[3 * j + k]);
    for (int k = 0; k < 3; ++k) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[k] = min(lo[k], (uint32_t)__shfl_xor((int)lo[k], o, 64));
            hi[k] = max(hi[k], (uint32_t)__shfl_xor((int)hi[k], o, 64));
        }
    }
    __shared__ uint32_t s_lo[4][3], s_hi[4][3];
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) {
            s_lo[threadIdx.x >> 6][k] = lo[k];
            s_hi[threadIdx.x >> 6][k] = hi[k];
        }
    __syncthreads();
    if (threadIdx.x < 3 && gb.g_end > gb.g_begin) {
        const int k = threadIdx.x;
        atomicMin(bb + 6 * gb.subject + k, min(min(s_lo[0][k], s_lo[1][k]), min(s_lo[2][k], s_lo[3][k])));
        atomicMax(bb + 6 * gb.subject + 3 + k, max(max(s_hi[0][k], s_hi[1][k]), max(s_hi[2][k], s_hi[3][k])));
    }
}

__global__ void k_cell_keys(const float* __restrict__ mean, const GaussBlock* __restrict__ blocks, int32_t nb,
                            const TopkGrid* __restrict__ grid, uint32_t* __restrict__ keys,
                            uint32_t* __restrict__ vals) {
    if ((int)blockIdx.x >= nb) return;
    const GaussBlock gb = blocks[blockIdx.x];
    const int64_t j = gb.g_begin + threadIdx.x;
    if (j >= gb.g_end) return;
    const TopkGrid& g = grid[gb.subject];
    int c[3];
    for (int k = 0; k < 3; ++k) {
        const int v = (int)floorf((mean[3 * j + k] - g.origin[k]) * g.inv_h);
        c[k] = min(max(v, 0), g.dims[k] - 1);
    }
    keys[j] = (uint32_t)(g.base + ((int64_t)c[2] * g.dims[1] + c[1]) * g.dims[0] + c[0]);
    vals[j] = (uint32_t)j;
}

__global__ void k_cell_ranges(const uint32_t* __restrict__ keys, int64_t n, int2* __restrict__ ranges,
                              uint32_t n_ranges) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t k = keys[s];
    if (k >= n_ranges) return;
    if (s == 0 || keys[s - 1] != k) ranges[k].x = (int)s;
    if (s == n - 1 || keys[s + 1] != k) ranges[k].y = (int)(s + 1);
}

// sorted means: (x, y, z, id bits)
__global__ void k_gather_means(const float* __restrict__ mean, const uint32_t* __restrict__ order, int64_t n,
                               float4* __restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t j = order[s];
    out[s] = make_float4(mean[3 * (int64_t)j], mean[3 * (int64_t)j + 1], mean[3 * (int64_t)j + 2],
                         __uint_as_float(j));
}

// --------------------------------------------------------------------------
// K nearest means per pixel
// --------------------------------------------------------------------------
struct KnnArgs {
    const SliceGeo* geo;
    const TopkSlice* slices;
    const TopkGrid* grid;
    const int2* cells;
    const float4* smean;     // means sorted by cell
    const float* mask;       // [P] or NULL: lists only for pixels with mask > 0
    int32_t K;
    int32_t* nbr;            // [P, K]; -1 where no list is built
    int* status;             // [2]: pixels that failed, sub-tile splits
};

__device__ inline int block_excl_scan_int(int v, int* s_wave, int& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
    for (int w = 0; w < kKnnThreads / 64; ++w) {
        if (w < wave) before += s_wave[w];
        total += s_wave[w];
    }
    __syncthreads();
    return before + incl - v;
}

struct KnnShared {
    float4 cand[kCandCap];
    uint16_t hist[kBins * kKnnThreads];
    int cell_off[kKnnThreads + 1];
    int cell_start[kKnnThreads];
    int wave[kKnnThreads / 64];
    int n;
    int box[4];
};

// Compacts into sh.cand, in cell order, the means within distance rho of the
// slice-frame rectangle [u0, u1] x [v0, v1] x {0} (a superset of the
// radius-rho balls of its pixels), keeping those whose compacted index lies
// in [lo, lo + kCandCap).  Returns the total count.  Block-uniform.
__device__ int gather_chunk(const KnnArgs& a, const TopkSlice& ts, const TopkGrid& g, float u0, float u1, float v0,
                            float v1, float rho, int lo, KnnShared& sh) {
    // world AABB of the rectangle grown by rho
    float blo[3] = {3.4e38f, 3.4e38f, 3.4e38f}, bhi[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
    for (int corner = 0; corner < 8; ++corner) {
        const float cu = (corner & 1) ? u1 + rho : u0 - rho;
        const float cv = (corner & 2) ? v1 + rho : v0 - rho;
        const float cz = (corner & 4) ? rho : -rho;
        for (int d = 0; d < 3; ++d) {
            const float w = fmaf(ts.R[3 * d], cu, fmaf(ts.R[3 * d + 1], cv, fmaf(ts.R[3 * d + 2], cz, ts.t[d])));
            blo[d] = fminf(blo[d], w);
            bhi[d] = fmaxf(bhi[d], w);
        }
    }
    int cl[3], ch[3];
    for (int d = 0; d < 3; ++d) {
        cl[d] = max((int)floorf((blo[d] - g.origin[d]) * g.inv_h), 0);
        ch[d] = min((int)floorf((bhi[d] - g.origin[d]) * g.inv_h), g.dims[d] - 1);
    }
    const int nx = ch[0] - cl[0] + 1, ny = ch[1] - cl[1] + 1, nz = ch[2] - cl[2] + 1;
    const int64_t ncell = (nx > 0 && ny > 0 && nz > 0) ? (int64_t)nx * ny * nz : 0;
    const float r2 = rho * rho;
    if (threadIdx.x == 0) sh.n = 0;
    __syncthreads();
    for (int64_t cb = 0; cb < ncell; cb += kKnnThreads) {
        const int64_t c = cb + threadIdx.x;
        int cnt = 0, start = 0;
        if (c < ncell) {
            const int cx = cl[0] + (int)(c % nx);
            const int cy = cl[1] + (int)((c / nx) % ny);
            const int cz = cl[2] + (int)(c / ((int64_t)nx * ny));
            const int2 rg = a.cells[g.base + ((int64_t)cz * g.dims[1] + cy) * g.dims[0] + cx];
            start = rg.x;
            cnt = rg.y - rg.x;
        }
        int total;
        const int off = block_excl_scan_int(cnt, sh.wave, total);
        sh.cell_off[threadIdx.x] = off;
        sh.cell_start[threadIdx.x] = start;
        __syncthreads();
        for (int qb = 0; qb < total; qb += kKnnThreads) {
            const int q = qb + threadIdx.x;
            bool keep = false;
            float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < total) {
                int l = 0, h = kKnnThreads - 1;   // last cell whose offset is <= q
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (sh.cell_off[mid] <= q) l = mid; else h = mid - 1;
                }
                m = a.smean[sh.cell_start[l] + (q - sh.cell_off[l])];
                const float dx = m.x - ts.t[0], dy = m.y - ts.t[1], dz = m.z - ts.t[2];
                const float mu = ts.R[0] * dx + ts.R[3] * dy + ts.R[6] * dz;
                const float mv = ts.R[1] * dx + ts.R[4] * dy + ts.R[7] * dz;
                const float mz = ts.R[2] * dx + ts.R[5] * dy + ts.R[8] * dz;
                const float du = fmaxf(fmaxf(u0 - mu, mu - u1), 0.f);
                const float dv = fmaxf(fmaxf(v0 - mv, mv - v1), 0.f);
                keep = du * du + dv * dv + mz * mz <= r2;
            }
            int kept;
            const int pos = block_excl_scan_int(keep ? 1 : 0, sh.wave, kept);
            const int idx = sh.n + pos - lo;
            if (keep && idx >= 0 && idx < kCandCap) sh.cand[idx] = m;
            __syncthreads();
            if (threadIdx.x == 0) sh.n += kept;
            __syncthreads();
        }
    }
    return sh.n;
}

__global__ __launch_bounds__(kKnnThreads) void k_knn(KnnArgs a) {
    __shared__ KnnShared sh;
    const int i = blockIdx.y;
    const SliceGeo& sg = a.geo[i];
    const int ntx = (sg.W + kKnnSide - 1) / kKnnSide, nty = (sg.H + kKnnSide - 1) / kKnnSide;
    if ((int)blockIdx.x >= ntx * nty) return;
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const TopkSlice& ts = a.slices[i];
    const TopkGrid& g = a.grid[sg.subject];
    const int lr = threadIdx.x / kKnnSide, lc = threadIdx.x % kKnnSide;
    const int r = ty * kKnnSide + lr, k = tx * kKnnSide + lc;
    const bool valid = r < sg.H && k < sg.W;
    float px, py, pz, ux, uy;
    pixel_world(sg, ts, min(r, sg.H - 1), min(k, sg.W - 1), px, py, pz, ux, uy);
    const int K = a.K;
    const int64_t pix = sg.pix_off + (int64_t)min(r, sg.H - 1) * sg.W + min(k, sg.W - 1);
    int32_t* out = a.nbr + pix * K;
    const bool need = valid && (!a.mask || a.mask[pix] > 0.f);
    if (valid && !need)
        for (int q = 0; q < K; ++q) out[q] = -1;
    if (!__syncthreads_or(need ? 1 : 0)) return;

    // Sub-tiles of side 8, 4, 2, then 1 while their candidates exceed LDS
    // (then they are streamed through LDS in chunks).  Each pixel finishes
    // as soon as it has K means within the current radius; the radius grows
    // (and the slab shrinks to the unfinished pixels) for the others only.
    bool fin = !need;
    for (int side = kKnnSide; side >= 1; side >>= 1) {
        const int nsub = kKnnSide / side;
        bool split = false;
        for (int sub = 0; sub < nsub * nsub && !split; ++sub) {
            const int sr = (sub / nsub) * side, sc = (sub % nsub) * side;
            const bool in_sub = need && lr >= sr && lr < sr + side && lc >= sc && lc < sc + side;
            float rho = 0.8f * g.rho0;
            for (int attempt = 0; attempt < kMaxTries; ++attempt, rho *= 1.3f) {
                const bool mine = in_sub && !fin;
                if (!__syncthreads_or(mine ? 1 : 0)) break;
                // pixel rectangle of the unfinished pixels
                if (threadIdx.x == 0) {
                    sh.box[0] = 1 << 30; sh.box[1] = -1; sh.box[2] = 1 << 30; sh.box[3] = -1;
                }
                __syncthreads();
                if (mine) {
                    atomicMin(&sh.box[0], r);
                    atomicMax(&sh.box[1], r);
                    atomicMin(&sh.box[2], k);
                    atomicMax(&sh.box[3], k);
                }
                __syncthreads();
                const int r0 = sh.box[0], r1 = sh.box[1], c0 = sh.box[2], c1 = sh.box[3];
                __syncthreads();
                const float u0 = ((float)c0 - 0.5f * (float)(sg.W - 1)) * sg.dx;
                const float u1 = ((float)c1 - 0.5f * (float)(sg.W - 1)) * sg.dx;
                const float v0 = ((float)r0 - 0.5f * (float)(sg.H - 1)) * sg.dy;
                const float v1 = ((float)r1 - 0.5f * (float)(sg.H - 1)) * sg.dy;
                const int n = gather_chunk(a, ts, g, u0, u1, v0, v1, rho, 0, sh);
                if (n > kCandCap && side > 1) {
                    split = true;
                    break;
                }
                const bool resident = n <= kCandCap;
                const int nch = (n + kCandCap - 1) / kCandCap;
                const float r2 = rho * rho;
                const float scale1 = (float)kBins / r2;
                // pass 1: histogram of squared distances over [0, rho^2)
                if (mine)
                    for (int b = 0; b < kBins; ++b) sh.hist[b * kKnnThreads + threadIdx.x] = 0;
                for (int chn = 0; chn < nch; ++chn) {
                    if (!resident) gather_chunk(a, ts, g, u0, u1, v0, v1, rho, chn * kCandCap, sh);
                    const int cnt = min(kCandCap, n - chn * kCandCap);
                    if (mine)
                        for (int c = 0; c < cnt; ++c) {
                            const float d2 = dist2(px, py, pz, sh.cand[c]);
                            if (d2 < r2) sh.hist[min((int)(d2 * scale1), kBins - 1) * kKnnThreads + threadIdx.x] += 1;
                        }
                    __syncthreads();
                }
                int have = 0, bstar = -1;
                if (mine) {
                    int cum = 0;
                    for (int b = 0; b < kBins; ++b) {
                        const int h = sh.hist[b * kKnnThreads + threadIdx.x];
                        if (cum + h >= K) { bstar = b; break; }
                        cum += h;
                    }
                    have = cum;
                }
                const bool res = mine && bstar >= 0;   // this pixel completes at this radius
                if (!__syncthreads_or(res ? 1 : 0)) continue;   // grow rho for all
                // pass 2: the boundary bin split into kBins sub-bins
                const float lo_b = res ? (float)bstar / scale1 : 0.f;
                const float scale2 = (float)kBins * scale1;
                if (res)
                    for (int b = 0; b < kBins; ++b) sh.hist[b * kKnnThreads + threadIdx.x] = 0;
                for (int chn = 0; chn < nch; ++chn) {
                    if (!resident) gather_chunk(a, ts, g, u0, u1, v0, v1, rho, chn * kCandCap, sh);
                    const int cnt = min(kCandCap, n - chn * kCandCap);
                    if (res)
                        for (int c = 0; c < cnt; ++c) {
                            const float d2 = dist2(px, py, pz, sh.cand[c]);
                            if (d2 < r2 && min((int)(d2 * scale1), kBins - 1) == bstar)
                                sh.hist[min(max((int)((d2 - lo_b) * scale2), 0), kBins - 1) * kKnnThreads + threadIdx.x] +=
                                    1;
                        }
                    __syncthreads();
                }
                int b2 = kBins - 1;
                if (res) {
                    int cum = have;
                    for (int b = 0; b < kBins; ++b) {
                        const int h = sh.hist[b * kKnnThreads + threadIdx.x];
                        if (cum + h >= K) { b2 = b; break; }
                        cum += h;
                    }
                }
                // pass 3: every mean below the boundary sub-bin, in candidate order
                int cnt_out = 0;
                for (int chn = 0; chn < nch; ++chn) {
                    if (!resident) gather_chunk(a, ts, g, u0, u1, v0, v1, rho, chn * kCandCap, sh);
                    const int cnt = min(kCandCap, n - chn * kCandCap);
                    if (res)
                        for (int c = 0; c < cnt; ++c) {
                            const float d2 = dist2(px, py, pz, sh.cand[c]);
                            if (d2 >= r2) continue;
                            const int b = min((int)(d2 * scale1), kBins - 1);
                            const bool take = b < bstar ||
                                              (b == bstar && min(max((int)((d2 - lo_b) * scale2), 0), kBins - 1) < b2);
                            if (take && cnt_out < K) out[cnt_out++] = (int32_t)__float_as_uint(sh.cand[c].w);
                        }
                    __syncthreads();
                }
                // exact picks inside the boundary sub-bin, by (d2, candidate index)
                float last_d = -1.f;
                int last_c = -1;
                bool stuck = false;
                while (__syncthreads_or(res && cnt_out < K && !stuck ? 1 : 0)) {
                    const bool want = res && cnt_out < K && !stuck;
                    float best_d = 3.4e38f;
                    int best_c = -1;
                    uint32_t best_id = 0;
                    for (int chn = 0; chn < nch; ++chn) {
                        if (!resident) gather_chunk(a, ts, g, u0, u1, v0, v1, rho, chn * kCandCap, sh);
                        const int cnt = min(kCandCap, n - chn * kCandCap);
                        if (want)
                            for (int c = 0; c < cnt; ++c) {
                                const float d2 = dist2(px, py, pz, sh.cand[c]);
                                if (d2 >= r2 || min((int)(d2 * scale1), kBins - 1) != bstar ||
                                    min(max((int)((d2 - lo_b) * scale2), 0), kBins - 1) != b2)
                                    continue;
                                const int gc = chn * kCandCap + c;
                                const bool after = d2 > last_d || (d2 == last_d && gc > last_c);
                                const bool better = d2 < best_d || (d2 == best_d && gc < best_c);
                                if (after && better) {
                                    best_d = d2;
                                    best_c = gc;
                                    best_id = __float_as_uint(sh.cand[c].w);
                                }
                            }
                        __syncthreads();
                    }
                    if (want) {
                        if (best_c < 0) {
                            stuck = true;
                        } else {
                            out[cnt_out++] = (int32_t)best_id;
                            last_d = best_d;
                            last_c = best_c;
                        }
                    }
                }
                if (res) {
                    if (cnt_out < K) {
                        for (int q = 0; q < K; ++q) out[q] = -1;
                        atomicAdd(a.status, 1);
                    }
                    fin = true;
                }
            }
            if (split) break;
            // radius limit reached without K means
            if (in_sub && !fin) {
                for (int q = 0; q < K; ++q) out[q] = -1;
                atomicAdd(a.status, 1);
                fin = true;
            }
            __syncthreads();
        }
        if (!split) return;
        if (threadIdx.x == 0) atomicAdd(a.status + 1, 1);
        __syncthreads();
    }
}

// (Gaussian, pixel) pairs of the neighbour lists
__global__ void k_pairs(const int32_t* __restrict__ lint, int64_t n, uint32_t* __restrict__ keys,
                        uint32_t* __restrict__ vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    keys[s] = (uint32_t)lint[s];   // cell-order position of the Gaussian
    vals[s] = (uint32_t)s;         // entry; its active pixel is s % n_act
}

__global__ void k_iperm(const uint32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ iperm) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) iperm[perm[s]] = (int32_t)s;
}

// Internal lists of the active pixels, entry t of active pixel a at
// lint[t * n_act + a] (coalesced over a wave's pixels), holding cell-order
// positions instead of ids.
__global__ void k_lists_internal(const int32_t* __restrict__ nbr, const int32_t* __restrict__ act, int64_t n_act,
                                 int32_t K, const int32_t* __restrict__ iperm, int32_t* __restrict__ lint) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_act * K) return;
    const int64_t t = e / n_act, a = e - t * n_act;
    lint[e] = iperm[nbr[(int64_t)act[a] * K + t]];
}

// Pixels with a list, in 8x8-patch order: position q of slice i enumerates
// its pixels padded to whole patches (patch row-major, then row-major inside
// the patch), so that consecutive listed pixels -- the lanes of a wave --
// form compact patches whose neighbour sets overlap.  qoff [M+1]: first
// position of each slice.
__device__ inline int64_t patch_pixel(const SliceGeo* geo, const int64_t* qoff, int32_t m, int64_t q, int& slice) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (qoff[mid] <= q) lo = mid; else hi = mid - 1;
    }
    slice = lo;
    const SliceGeo& sg = geo[lo];
    const int64_t l = q - qoff[lo];
    const int ntx8 = (sg.W + 7) >> 3;
    const int64_t pi = l >> 6;
    const int w = (int)(l & 63);
    const int y = (int)(pi / ntx8) * 8 + (w >> 3), x = (int)(pi % ntx8) * 8 + (w & 7);
    return (y < sg.H && x < sg.W) ? sg.pix_off + (int64_t)y * sg.W + x : -1;
}

__global__ void k_act_flags(const int32_t* __restrict__ nbr, const SliceGeo* __restrict__ geo,
                            const int64_t* __restrict__ qoff, int32_t m, int64_t Q, int32_t K, int* __restrict__ flag,
                            uint8_t* __restrict__ active) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    int slice;
    const int64_t p = patch_pixel(geo, qoff, m, q, slice);
    const int f = (p >= 0 && nbr[p * K] >= 0) ? 1 : 0;
    flag[q] = f;
    if (p >= 0) active[p] = (uint8_t)f;
}

__global__ void k_act_compact(const int* __restrict__ flag, const int* __restrict__ off, const SliceGeo* __restrict__ geo,
                              const int64_t* __restrict__ qoff, int32_t m, int64_t Q, int32_t* __restrict__ act) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q || !flag[q]) return;
    int slice;
    act[off[q]] = (int32_t)patch_pixel(geo, qoff, m, q, slice);
}

__global__ void k_act_offsets(const int* __restrict__ off, const int64_t* __restrict__ qoff, int32_t m,
                              const long long* __restrict__ total, int32_t* __restrict__ act_off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > m) return;
    act_off[i] = i < m ? off[qoff[i]] : (int32_t)total[0];
}

// --------------------------------------------------------------------------
// forward
// --------------------------------------------------------------------------
struct TopkFwdArgs {
    const SliceGeo* geo;
    const TopkSlice* slices;
    const TopkGauss* gauss;
    const int32_t* nbr;       // internal lists [n_act, K] (cell-order positions)
    const int32_t* act;       // pixels with a list, increasing
    const int32_t* act_off;   // [M+1] each slice's range in act
    int64_t n_act;
    int32_t K;
    float delta;
    int32_t loss_kind;
};

// Pixels without a list: prediction 0 and their data term (pixels of the
// build's mask all have lists, so with that mask these terms are 0).
__global__ __launch_bounds__(kBlock) void k_topk_inactive(const SliceGeo* __restrict__ geo,
                                                          const uint8_t* __restrict__ active, int32_t loss_kind,
                                                          const float* __restrict__ target,
                                                          const float* __restrict__ mask,
                                                          const float* __restrict__ msum, float* __restrict__ pred,
                                                          float* __restrict__ grad, float* __restrict__ partial,
                                                          int32_t blocks_x, int32_t stride) {
    __shared__ float s_red[kBlock / 64];
    const int i = blockIdx.y;
    const SliceGeo& sg = geo[i];
    const int64_t n = (int64_t)sg.H * sg.W;
    const float inv_msum = (msum && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float acc = 0.f;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)blocks_x * kBlock) {
        const int64_t p = sg.pix_off + q;
        if (active[p]) continue;
        pred[p] = 0.f;
        if (target) {
            const float m = mask ? mask[p] : 1.f;
            const float rr = -target[p];
            if (loss_kind == 0) {
                acc = fmaf(m * rr, rr, acc);
                if (grad) grad[p] = 2.f * m * rr * inv_msum;
            } else {
                acc = fmaf(m, fabsf(rr), acc);
                if (grad) grad[p] = rr > 0.f ? m : (rr < 0.f ? -m : 0.f);
            }
        }
    }
    if (!partial) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)i * stride + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// One thread per pixel with a list; act [n_act] holds those pixels in
// increasing order, act_off [M+1] each slice's range in it.
__global__ __launch_bounds__(kBlock) void k_topk_forward(TopkFwdArgs a, const float* __restrict__ target,
                                                         const float* __restrict__ mask,
                                                         const float* __restrict__ msum, float* __restrict__ pred,
                                                         float2* __restrict__ state, float* __restrict__ grad,
                                                         float* __restrict__ partial, int32_t blocks_x,
                                                         int32_t stride) {
    __shared__ float s_red[kBlock / 64];
    const int i = blockIdx.y;
    const SliceGeo& sg = a.geo[i];
    const TopkSlice& ts = a.slices[i];
    const int a0 = a.act_off[i], a1 = a.act_off[i + 1];
    const float inv_msum = (msum && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float acc = 0.f;
    for (int qa = a0 + blockIdx.x * kBlock + threadIdx.x; qa < a1; qa += blocks_x * kBlock) {
        const int64_t p = a.act[qa];
        const int64_t q = p - sg.pix_off;
        const int r = (int)(q / sg.W), k = (int)(q - (int64_t)r * sg.W);
        float x, y, z, ux, uy;
        pixel_world(sg, ts, r, k, x, y, z, ux, uy);
        const int32_t* nb = a.nbr + qa;
        float num = 0.f, den = 0.f;
        for (int t = 0; t < a.K; ++t) {
            const TopkGauss g = a.gauss[nb[(int64_t)t * a.n_act]];
            const float S[6] = {g.b.x + ts.P[0], g.b.y + ts.P[1], g.b.z + ts.P[2],
                                g.b.w + ts.P[3], g.c.x + ts.P[4], g.c.y + ts.P[5]};
            float wx, wy, wz;
            const float e = pair_eval(S, x - g.a.x, y - g.a.y, z - g.a.z, wx, wy, wz);
            num = fmaf(g.a.w, e, num);
            den += e;
        }
        const float dd = den + a.delta;
        const float yn = num / dd;
        const float yv = ts.sigma * yn;
        pred[p] = yv;
        if (state) state[qa] = make_float2(yn, dd);
        if (target) {
            const float m = mask ? mask[p] : 1.f;
            const float rr = yv - target[p];
            if (a.loss_kind == 0) {
                acc = fmaf(m * rr, rr, acc);
                if (grad) grad[p] = 2.f * m * rr * inv_msum;
            } else {
                acc = fmaf(m, fabsf(rr), acc);
                if (grad) grad[p] = rr > 0.f ? m : (rr < 0.f ? -m : 0.f);
            }
        }
    }
    if (!partial) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)i * stride + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ __launch_bounds__(kBlock) void k_topk_loss(const float* __restrict__ partial, int64_t n,
                                                      const float* __restrict__ msum, int32_t kind,
                                                      float* __restrict__ loss) {
    __shared__ float s[kBlock / 64];
    float acc = 0.f;
    for (int64_t q = threadIdx.x; q < n; q += kBlock) acc += partial[q];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = s[0] + s[1] + s[2] + s[3];
        if (kind == 0) loss[0] = (msum && msum[0] > 0.f) ? tot / msum[0] : 0.f;
        else loss[0] = tot;
    }
}

// --------------------------------------------------------------------------
// adjoint
// --------------------------------------------------------------------------
constexpr int kPoseTerms = 13;   // (R u) x dx (3), dx (3), G_P (6), d sigma (1)

// Also leaves, per listed pixel, what the Gaussian pass needs: pxw = (x, gs)
// with gs = g sigma / (D + delta) (0: skip), pyd = (N / (D + delta), slice).
__global__ __launch_bounds__(kBlock) void k_topk_pose_pass(TopkFwdArgs a, const float* __restrict__ grad_pred,
                                                           const float2* __restrict__ state,
                                                           float* __restrict__ partial, int32_t blocks_x,
                                                           float4* __restrict__ pxw, float2* __restrict__ pyd) {
    __shared__ float s_red[kPoseTerms][kBlock / 64];
    const int i = blockIdx.y;
    const SliceGeo& sg = a.geo[i];
    const TopkSlice& ts = a.slices[i];
    const int a0 = a.act_off[i], a1 = a.act_off[i + 1];
    float acc[kPoseTerms];
    for (int e = 0; e < kPoseTerms; ++e) acc[e] = 0.f;
    for (int qa = a0 + blockIdx.x * kBlock + threadIdx.x; qa < a1; qa += blocks_x * kBlock) {
        const int64_t p = a.act[qa];
        const float gy = grad_pred[p];
        const int64_t q = p - sg.pix_off;
        const int r = (int)(q / sg.W), k = (int)(q - (int64_t)r * sg.W);
        float x, y, z, ux, uy;
        pixel_world(sg, ts, r, k, x, y, z, ux, uy);
        const float2 st = state[qa];
        const float yn = st.x, inv_dd = 1.f / st.y;
        const float gs = gy * ts.sigma * inv_dd;
        pxw[qa] = make_float4(x, y, z, gs);
        pyd[qa] = make_float2(yn, __int_as_float(i));
        if (gy == 0.f) continue;
        const int32_t* nb = a.nbr + qa;
        float dx0 = 0.f, dx1 = 0.f, dx2 = 0.f;
        float G[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < a.K; ++t) {
            const TopkGauss g = a.gauss[nb[(int64_t)t * a.n_act]];
            const float S[6] = {g.b.x + ts.P[0], g.b.y + ts.P[1], g.b.z + ts.P[2],
                                g.b.w + ts.P[3], g.c.x + ts.P[4], g.c.y + ts.P[5]};
            float wx, wy, wz;
            const float e = pair_eval(S, x - g.a.x, y - g.a.y, z - g.a.z, wx, wy, wz);
            const float ge = gs * (g.a.w - yn) * e;      // dL/de * e
            dx0 -= ge * wx;
            dx1 -= ge * wy;
            dx2 -= ge * wz;
            const float h = 0.5f * ge;
            G[0] = fmaf(h * wx, wx, G[0]);
            G[1] = fmaf(h * wx, wy, G[1]);
            G[2] = fmaf(h * wx, wz, G[2]);
            G[3] = fmaf(h * wy, wy, G[3]);
            G[4] = fmaf(h * wy, wz, G[4]);
            G[5] = fmaf(h * wz, wz, G[5]);
        }
        // R u (world offset of the pixel from the slice centre)
        const float ru0 = ts.R[0] * ux + ts.R[1] * uy, ru1 = ts.R[3] * ux + ts.R[4] * uy,
                    ru2 = ts.R[6] * ux + ts.R[7] * uy;
        acc[0] += ru1 * dx2 - ru2 * dx1;
        acc[1] += ru2 * dx0 - ru0 * dx2;
        acc[2] += ru0 * dx1 - ru1 * dx0;
        acc[3] += dx0;
        acc[4] += dx1;
        acc[5] += dx2;
        for (int e = 0; e < 6; ++e) acc[6 + e] += G[e];
        acc[12] += gy * yn;
    }
    for (int e = 0; e < kPoseTerms; ++e) {
        float v = acc[e];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) s_red[e][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < kPoseTerms) {
        const int e = threadIdx.x;
        partial[((int64_t)i * blocks_x + blockIdx.x) * kPoseTerms + e] =
            s_red[e][0] + s_red[e][1] + s_red[e][2] + s_red[e][3];
    }
}

// Per slice: sums of the block partials -> pose accumulator (d delta, d tau)
// and d sigma.
__global__ void k_topk_pose_reduce(const float* __restrict__ partial, int32_t blocks_x,
                                   const TopkSlice* __restrict__ slices, int32_t m, float* __restrict__ pose_acc,
                                   float* __restrict__ g_sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float s[kPoseTerms];
    for (int e = 0; e < kPoseTerms; ++e) s[e] = 0.f;
    for (int b = 0; b < blocks_x; ++b)
        for (int e = 0; e < kPoseTerms; ++e) s[e] += partial[((int64_t)i * blocks_x + b) * kPoseTerms + e];
    // PSF term of the left perturbation: A = P G, d delta += 2 (A12 - A21, A20 - A02, A01 - A10)
    const float* P = slices[i].P;
    const float Pm[9] = {P[0], P[1], P[2], P[1], P[3], P[4], P[2], P[4], P[5]};
    const float Gm[9] = {s[6], s[7], s[8], s[7], s[9], s[10], s[8], s[10], s[11]};
    float A[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            A[3 * r + c] = Pm[3 * r] * Gm[c] + Pm[3 * r + 1] * Gm[3 + c] + Pm[3 * r + 2] * Gm[6 + c];
    pose_acc[6 * i + 0] = s[0] + 2.f * (A[5] - A[7]);
    pose_acc[6 * i + 1] = s[1] + 2.f * (A[6] - A[2]);
    pose_acc[6 * i + 2] = s[2] + 2.f * (A[1] - A[3]);
    pose_acc[6 * i + 3] = s[3];
    pose_acc[6 * i + 4] = s[4];
    pose_acc[6 * i + 5] = s[5];
    if (g_sigma) g_sigma[i] = s[12];
}

// One wave per Gaussian over the pixels whose lists hold it.
__global__ __launch_bounds__(kBlock) void k_topk_gauss_pass(
        TopkFwdArgs a, const int2* __restrict__ granges, const uint32_t* __restrict__ gpix,
        const uint32_t* __restrict__ perm, const float4* __restrict__ pxw, const float2* __restrict__ pyd,
        const float* __restrict__ log_scale, const float* __restrict__ quat, int64_t n_gauss,
        float* __restrict__ g_mean, float* __restrict__ g_ls, float* __restrict__ g_quat,
        float* __restrict__ g_amp) {
    const int64_t pos = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (pos >= n_gauss) return;
    const int64_t j = perm[pos];
    const TopkGauss g = a.gauss[pos];
    const int2 rg = granges[pos];
    float acc[10];
    for (int e = 0; e < 10; ++e) acc[e] = 0.f;
    for (int s = rg.x + lane; s < rg.y; s += 64) {
        const int64_t ai = (int64_t)gpix[s] % a.n_act;
        const float4 xw = pxw[ai];
        const float gs = xw.w;
        if (gs == 0.f) continue;
        const float2 yd = pyd[ai];
        const float* P = a.slices[__float_as_int(yd.y)].P;
        const float S[6] = {g.b.x + P[0], g.b.y + P[1], g.b.z + P[2], g.b.w + P[3], g.c.x + P[4], g.c.y + P[5]};
        float wx, wy, wz;
        const float e = pair_eval(S, xw.x - g.a.x, xw.y - g.a.y, xw.z - g.a.z, wx, wy, wz);
        acc[0] += gs * e;                       // d c
        const float ge = gs * (g.a.w - yd.x) * e;
        acc[1] += ge * wx;                      // d mu
        acc[2] += ge * wy;
        acc[3] += ge * wz;
        const float h = 0.5f * ge;              // d Sigma (full-matrix gradient, symmetric)
        acc[4] = fmaf(h * wx, wx, acc[4]);
        acc[5] = fmaf(h * wx, wy, acc[5]);
        acc[6] = fmaf(h * wx, wz, acc[6]);
        acc[7] = fmaf(h * wy, wy, acc[7]);
        acc[8] = fmaf(h * wy, wz, acc[8]);
        acc[9] = fmaf(h * wz, wz, acc[9]);
    }
    for (int e = 0; e < 10; ++e)
        for (int o = 32; o > 0; o >>= 1) acc[e] += __shfl_xor(acc[e], o, 64);
    if (lane != 0) return;
    g_amp[j] = acc[0];
    g_mean[3 * j] = acc[1];
    g_mean[3 * j + 1] = acc[2];
    g_mean[3 * j + 2] = acc[3];
    // Sigma = R diag(s^2) R^T: d log s_k = 2 s_k^2 (R^T G R)_kk, dR = 2 G R diag(s^2)
    const float Gm[9] = {acc[4], acc[5], acc[6], acc[5], acc[7], acc[8], acc[6], acc[8], acc[9]};
    const float qn = sqrtf(quat[4 * j] * quat[4 * j] + quat[4 * j + 1] * quat[4 * j + 1] +
                           quat[4 * j + 2] * quat[4 * j + 2] + quat[4 * j + 3] * quat[4 * j + 3]);
    const float w = quat[4 * j] / qn, x = quat[4 * j + 1] / qn, y = quat[4 * j + 2] / qn, z = quat[4 * j + 3] / qn;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    float s2[3];
    for (int k = 0; k < 3; ++k) s2[k] = expf(2.f * log_scale[3 * j + k]);
    float GR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GR[3 * r + c] = Gm[3 * r] * R[c] + Gm[3 * r + 1] * R[3 + c] + Gm[3 * r + 2] * R[6 + c];
    for (int k = 0; k < 3; ++k) {
        const float rgr = R[k] * GR[k] + R[3 + k] * GR[3 + k] + R[6 + k] * GR[6 + k];
        g_ls[3 * j + k] = 2.f * s2[k] * rgr;
    }
    float dR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dR[3 * r + c] = 2.f * GR[3 * r + c] * s2[c];
    // dR/d(w, x, y, z) of the unit quaternion
    const float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    const float dx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                            w * dR[7] - 2.f * x * dR[8]);
    const float dy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                            z * dR[7] - 2.f * y * dR[8]);
    const float dz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                            x * dR[6] + y * dR[7]);
    const float dot = w * dw + x * dx + y * dy + z * dz;
    g_quat[4 * j] = (dw - w * dot) / qn;
    g_quat[4 * j + 1] = (dx - x * dot) / qn;
    g_quat[4 * j + 2] = (dy - y * dot) / qn;
    g_quat[4 * j + 3] = (dz - z * dot) / qn;
}

}  // namespace

hipError_t launch_topk_prepare(const float* mean, const float* log_scale, const float* quat, const float* amp,
                               int64_t n, const uint32_t* perm, const SlicePose* pose, const SliceGeo* geo,
                               const float* sigma, int32_t m, TopkGauss* gauss, TopkSlice* slices, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_topk_activate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mean, log_scale,
                           quat, amp, n, perm, gauss);
    if (m > 0) hipLaunchKernelGGL(k_topk_slices, dim3((m + 127) / 128), dim3(128), 0, st, pose, geo, sigma, m, slices);
    return hipGetLastError();
}

hipError_t launch_topk_bbox(const float* mean, const GaussBlock* blocks, int32_t nb, int32_t n_subjects,
                            uint32_t* bb, hipStream_t st) {
    for (int s = 0; s < n_subjects; ++s) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, bb + 6 * s, (int64_t)3, 0xffffffffu);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, bb + 6 * s + 3, (int64_t)3, 0u);
    }
    if (nb > 0) hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, st, mean, blocks, nb, bb);
    return hipGetLastError();
}

float topk_order_float(uint32_t k) {
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

hipError_t launch_topk_cells(const float* mean, const GaussBlock* blocks, int32_t nb, const TopkGrid* grid,
                             int64_t n, int64_t n_cells, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, void* sort_tmp, int key_bits, int2* cells, float4* smean,
                             const uint32_t** perm, hipStream_t st) {
    if (nb > 0) hipLaunchKernelGGL(k_cell_keys, dim3(nb), dim3(256), 0, st, mean, blocks, nb, grid, keys, vals);
    bool alt = false;
    hipError_t e = launch_radix_sort(keys, vals, keys_alt, vals_alt, n, key_bits, sort_tmp, &alt, st);
    if (e != hipSuccess) return e;
    const uint32_t* sk = alt ? keys_alt : keys;
    const uint32_t* sv = alt ? vals_alt : vals;
    *perm = sv;
    e = launch_fill_zero(cells, sizeof(int2) * (size_t)n_cells, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sk, n, cells,
                           (uint32_t)n_cells);
        hipLaunchKernelGGL(k_gather_means, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mean, sv, n, smean);
    }
    return hipGetLastError();
}

int32_t topk_knn_tiles(int32_t H, int32_t W) { return ((W + kKnnSide - 1) / kKnnSide) * ((H + kKnnSide - 1) / kKnnSide); }

hipError_t launch_topk_knn(const SliceGeo* geo, const TopkSlice* slices, const TopkGrid* grid, const int2* cells,
                           const float4* smean, const float* mask, int32_t m, int32_t max_tiles, int32_t K,
                           int32_t* nbr, int* status, hipStream_t st) {
    if (m <= 0 || max_tiles <= 0) return hipSuccess;
    KnnArgs a{geo, slices, grid, cells, smean, mask, K, nbr, status};
    hipLaunchKernelGGL(k_knn, dim3(max_tiles, m), dim3(kKnnThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_topk_internal(const int32_t* nbr, const int32_t* act, int64_t n_act, int32_t K,
                                const uint32_t* perm, int64_t n_gauss, int32_t* iperm, int32_t* lint, hipStream_t st) {
    if (n_gauss > 0)
        hipLaunchKernelGGL(k_iperm, dim3((unsigned)((n_gauss + 255) / 256)), dim3(256), 0, st, perm, n_gauss, iperm);
    const int64_t n = n_act * K;
    if (n > 0)
        hipLaunchKernelGGL(k_lists_internal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nbr, act, n_act, K,
                           (const int32_t*)iperm, lint);
    return hipGetLastError();
}

hipError_t launch_topk_inverse(const int32_t* lint, int64_t n_pairs, int64_t n_gauss, int key_bits,
                               uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                               void* sort_tmp, int2* granges, const uint32_t** gpix, hipStream_t st) {
    if (n_pairs > 0)
        hipLaunchKernelGGL(k_pairs, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, st, lint, n_pairs, keys,
                           vals);
    bool alt = false;
    hipError_t e = launch_radix_sort(keys, vals, keys_alt, vals_alt, n_pairs, key_bits, sort_tmp, &alt, st);
    if (e != hipSuccess) return e;
    const uint32_t* sk = alt ? keys_alt : keys;
    *gpix = alt ? vals_alt : vals;
    e = launch_fill_zero(granges, sizeof(int2) * (size_t)n_gauss, st);
    if (e != hipSuccess) return e;
    if (n_pairs > 0)
        hipLaunchKernelGGL(k_cell_ranges, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, st, sk, n_pairs,
                           granges, (uint32_t)n_gauss);
    return hipGetLastError();
}

int32_t topk_blocks_x(int32_t max_hw) { return std::max(1, std::min((max_hw + kBlock - 1) / kBlock, 64)); }

hipError_t launch_topk_active(const int32_t* nbr, int32_t K, const SliceGeo* geo, const int64_t* qoff, int32_t m,
                              int64_t Q, int* flag, int* off, uint8_t* active, int32_t* act, int32_t* act_off,
                              long long* total, void* scan_tmp, hipStream_t st) {
    if (Q <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((Q + 255) / 256);
    hipLaunchKernelGGL(k_act_flags, dim3(nb), dim3(256), 0, st, nbr, geo, qoff, m, Q, K, flag, active);
    hipError_t e = launch_scan_int(flag, off, Q, total, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_act_compact, dim3(nb), dim3(256), 0, st, (const int*)flag, (const int*)off, geo, qoff, m, Q,
                       act);
    hipLaunchKernelGGL(k_act_offsets, dim3((m + 1 + 63) / 64), dim3(64), 0, st, (const int*)off, qoff, m,
                       (const long long*)total, act_off);
    return hipGetLastError();
}

size_t topk_loss_partial_floats(int32_t m, int32_t max_hw, int32_t max_act) {
    return (size_t)m * (topk_blocks_x(max_hw) + topk_blocks_x(max_act));
}

hipError_t launch_topk_forward(const SliceGeo* geo, const TopkSlice* slices, const TopkGauss* gauss,
                               const int32_t* nbr, const int32_t* act, const int32_t* act_off, const uint8_t* active,
                               int64_t n_act, int32_t K, float delta, int32_t loss_kind, int32_t m, int32_t max_hw, int32_t max_act,
                               const float* target, const float* mask, const float* msum, float* pred, float2* state,
                               float* grad, float* partial, float* loss, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    TopkFwdArgs a{geo, slices, gauss, nbr, act, act_off, n_act, K, delta, loss_kind};
    const int bx = topk_blocks_x(max_hw), ba = topk_blocks_x(max_act);
    const bool want = target && loss;
    hipLaunchKernelGGL(k_topk_inactive, dim3(bx, m), dim3(kBlock), 0, st, geo, active, loss_kind, target, mask, msum,
                       pred, grad, want ? partial : nullptr, bx, bx + ba);
    hipLaunchKernelGGL(k_topk_forward, dim3(ba, m), dim3(kBlock), 0, st, a, target, mask, msum, pred, state, grad,
                       want ? partial + bx : nullptr, ba, bx + ba);
    if (want)
        hipLaunchKernelGGL(k_topk_loss, dim3(1), dim3(kBlock), 0, st, (const float*)partial,
                           (int64_t)m * (bx + ba), msum, loss_kind, loss);
    return hipGetLastError();
}

size_t topk_pose_partial_floats(int32_t m, int32_t max_act) {
    return (size_t)m * topk_blocks_x(max_act) * kPoseTerms;
}

hipError_t launch_topk_backward(const SliceGeo* geo, const TopkSlice* slices, const TopkGauss* gauss,
                                const int32_t* nbr, const int32_t* act, const int32_t* act_off, int64_t n_act,
                                int32_t K, int32_t m, int32_t max_act, const float* grad_pred, const float2* state, const int2* granges,
                                const uint32_t* gpix, const uint32_t* perm, const float* log_scale, const float* quat,
                                int64_t n_gauss,
                                float* g_mean, float* g_ls, float* g_quat, float* g_amp, float* partial,
                                float* pose_acc, float* g_sigma, float4* pxw, float2* pyd, hipStream_t st) {
    TopkFwdArgs a{geo, slices, gauss, nbr, act, act_off, n_act, K, 0.f, 0};
    if (m > 0) {
        const int bx = topk_blocks_x(max_act);
        hipLaunchKernelGGL(k_topk_pose_pass, dim3(bx, m), dim3(kBlock), 0, st, a, grad_pred, state, partial, bx, pxw,
                           pyd);
        hipLaunchKernelGGL(k_topk_pose_reduce, dim3((m + 63) / 64), dim3(64), 0, st, (const float*)partial, bx,
                           slices, m, pose_acc, g_sigma);
    }
    if (n_gauss > 0)
        hipLaunchKernelGGL(k_topk_gauss_pass, dim3((unsigned)((n_gauss * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           st, a, granges, gpix, perm, (const float4*)pxw, (const float2*)pyd, log_scale, quat,
                           n_gauss, g_mean, g_ls, g_quat, g_amp);
    return hipGetLastError();
}

}  // namespace svr
