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
// Forward, record per lane (the alternative mode): each lane owns one instance
// and walks its record's footprint box inside the tile, accumulating into an
// LDS pixel tile with ds_add_f32; only box pixels are evaluated.
//
// Adjoint (record per lane): a workgroup takes a fixed chunk of 256 instances
// of the tile-ordered list and stages the upstream gradients of the chunk's
// tiles in LDS; each lane owns one instance and walks the pixels of its
// record's footprint box inside its tile, accumulating the seven moment sums
// it needs in registers (no cross-lane reduction), and writes them to the
// instance's emission slot (no atomics).
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
    const uint32_t k = keys[s] >> kClassBits;  // tile id
    if (k >= n_tiles) return;
    if (s == 0 || (keys[s - 1] >> kClassBits) != k) ranges[k].x = (int)s;
    if (s == n - 1 || (keys[s + 1] >> kClassBits) != k) ranges[k].y = (int)(s + 1);
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

// Per-pixel data term of the loss (r = y - I, mask m): kind 0 the masked mean
// squared error (m r^2, gradient 2 m r / sum m), kind 1 the masked L1 term of
// Eq. 7 (m |r|, subgradient m sign r, 0 at r = 0).
__device__ inline void loss_term(int kind, float m, float r, float inv_msum, float& acc, float* gp) {
    if (kind == 0) {
        acc = fmaf(m * r, r, acc);
        if (gp) *gp = 2.f * m * r * inv_msum;
    } else {
        acc = fmaf(m, fabsf(r), acc);
        if (gp) *gp = r > 0.f ? m : (r < 0.f ? -m : 0.f);
    }
}

// loss = sum of the per-slice sums, divided by the mask sum (msum != NULL) or not.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ slice_sse, int m,
                                              const float* __restrict__ msum, float* __restrict__ loss) {
    __shared__ float s[4];
    float acc = 0.f;
    for (int i = threadIdx.x; i < m; i += blockDim.x) acc += slice_sse[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = s[0] + s[1] + s[2] + s[3];
        if (msum) {
            const float ms = msum[0];
            loss[0] = ms > 0.f ? tot / ms : 0.f;
        } else {
            loss[0] = tot;
        }
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

// Origin of a tile from the per-tile table (static geometry): global pixel
// id of its first pixel, tile-local clip (valid width and height) and the
// slice width.
struct TileOrg {
    int64_t base;
    int x0, y0, stride, vw, vh;
};

__device__ inline TileOrg tile_org(int4 v) {
    TileOrg o;
    o.base = (int64_t)(((uint64_t)(uint32_t)v.y << 32) | (uint64_t)(uint32_t)v.x);
    o.x0 = v.z & 0xffff;
    o.y0 = (int)((uint32_t)v.z >> 16);
    o.stride = v.w & 0xffff;
    o.vw = (v.w >> 16) & 0xff;
    o.vh = (int)((uint32_t)v.w >> 24);
    return o;
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
                    loss_term(a.loss_kind, m, r, inv_msum, sq, grad ? grad + pi : nullptr);
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

// Footprint box of one record inside one tile, for record-per-lane kernels.
struct LaneBox {
    float pxl, pyl;             // record centre in tile-local pixel coordinates
    float bz, am, a00, a01, a11;
    int x0, x1, y0, y1;         // inclusive tile-local box, empty if x0 > x1 or y0 > y1
};

__device__ inline LaneBox lane_box(const Record& R, int tx0, int ty0, int xmax, int ymax, float tau2k) {
    LaneBox b;
    b.pxl = R.r0.x - (float)tx0;
    b.pyl = R.r0.y - (float)ty0;
    b.bz = R.r0.z;
    b.am = R.r0.w;
    b.a00 = R.r1.x;
    b.a01 = R.r1.y;
    b.a11 = R.r1.z;
    const float det = b.a00 * b.a11 - b.a01 * b.a01;
    const float rk = tau2k - b.bz;  // KZ (T^2 - beta) <= 0 inside the footprint
    // hardware reciprocal and square root (about 1 ulp each): the 1e-3 px
    // slack keeps the box conservative
    const float rkd = rk * __builtin_amdgcn_rcpf(det);
    const float hx = __builtin_amdgcn_sqrtf(fmaxf(rkd * b.a11, 0.f)) + 1e-3f;
    const float hy = __builtin_amdgcn_sqrtf(fmaxf(rkd * b.a00, 0.f)) + 1e-3f;
    // clamp in float before converting (the centre can be far outside the tile)
    b.x0 = (int)fmaxf(ceilf(b.pxl - hx), 0.f);
    b.x1 = (int)fminf(floorf(b.pxl + hx), (float)xmax);
    b.y0 = (int)fmaxf(ceilf(b.pyl - hy), 0.f);
    b.y1 = (int)fminf(floorf(b.pyl + hy), (float)ymax);
    return b;
}

// Forward, record per lane, persistent grid (persistent = 1): workgroups pull
// whole tiles heaviest-first from a work queue, with exact integer
// accumulation.  Per round of up to 256 of the tile's instances: the boxes
// are counting-sorted by shape in LDS (a wave's lanes then walk boxes of one
// shape), each lane walks one box
// rows outer / columns inner and adds round(a max(e - e_T, 0) / quantum) to
// the pixel's int32 LDS sum with an integer LDS atomic (float LDS atomics are
// slow on this GPU, integer ones are not).  The quantum is 2^(e - 30) with
// 2^e above the round's sum of |a|, so no pixel's round sum can overflow and
// the rounding error per term is below 2^-31 of that sum.  Integer sums do
// not depend on the order of the adds; each pixel's owner thread then adds
// the round's total to its float sum in round order, so the result is
// deterministic.
template <int T, bool kLoss, bool kCount>
__global__ __launch_bounds__(256) void k_forward_rpl_tiles(RenderArgs a, const float* __restrict__ target,
                                                     const float* __restrict__ mask,
                                                     const float* __restrict__ msum,
                                                     float* __restrict__ pred, float* __restrict__ grad,
                                                     float* __restrict__ tile_sse,
                                                     unsigned long long* __restrict__ incut,
                                                     int* __restrict__ work_counter) {
    constexpr int NT = 256, NW = 4;
    constexpr int kB = (T + 1) * (T + 1);
    __shared__ float s_acc[T * T];
    __shared__ int s_iacc[T * T];
    __shared__ float4 s_box[NT][2];
    __shared__ int s_hist[kB];
    __shared__ int s_perm[NT];
    __shared__ int s_wsum[NW];
    __shared__ float s_fsum[NW];
    __shared__ float s_red[NW];
    __shared__ unsigned int s_cnt[NW];
    __shared__ int s_next;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile < 0) break;
        const TileCoord tc = tile_coord(a, tile);
        const int2 rg = a.ranges[tile];
        const int xmax = min(T, tc.W - tc.x0) - 1, ymax = min(T, tc.H - tc.y0) - 1;
        __syncthreads();
        for (int p = tid; p < T * T; p += NT) {
            s_acc[p] = 0.f;
            s_iacc[p] = 0;
        }
        unsigned int cnt = 0;
        const int n = rg.y - rg.x;
        for (int r0 = 0; r0 < n; r0 += NT) {
            const int nb = min(NT, n - r0);
            for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
            __syncthreads();
            int bucket = 0, pos = 0;
            float absa = 0.f;
            if (tid < nb) {
                const Record R = a.rec[a.inst_rec[rg.x + r0 + tid]];
                const LaneBox b = lane_box(R, tc.x0, tc.y0, xmax, ymax, tau2k);
                const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
                const bool empty = w == 0 || h == 0;
                const int x0 = empty ? 0 : b.x0, x1 = empty ? -1 : b.x1;
                const int y0 = empty ? 0 : b.y0, y1 = empty ? -1 : b.y1;
                bucket = empty ? 0 : (h * (T + 1) + w);
                absa = empty ? 0.f : fabsf(b.am);
                s_box[tid][0] = make_float4(b.pxl, b.pyl, b.bz, b.am);
                s_box[tid][1] = make_float4(b.a00, b.a01, b.a11,
                                            __int_as_float((x0 + 1) | ((x1 + 1) << 8) | ((y0 + 1) << 16) |
                                                           ((y1 + 1) << 24)));
                pos = atomicAdd(&s_hist[bucket], 1);
            }
            for (int o = 32; o > 0; o >>= 1) absa += __shfl_xor(absa, o, 64);
            if (lane == 0) s_fsum[wv] = absa;
            __syncthreads();
            const float suma = (s_fsum[0] + s_fsum[1]) + (s_fsum[2] + s_fsum[3]);
            {
                const int per = (kB + NT - 1) / NT;
                const int kb = min(tid * per, kB), ke = min(kb + per, kB);
                int local = 0;
                for (int k = kb; k < ke; ++k) local += s_hist[k];
                int incl = local;
                for (int o = 1; o < 64; o <<= 1) {
                    const int u = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += u;
                }
                if (lane == 63) s_wsum[wv] = incl;
                __syncthreads();
                int run = incl - local;
                for (int q = 0; q < wv; ++q) run += s_wsum[q];
                for (int k = kb; k < ke; ++k) {
                    const int c = s_hist[k];
                    s_hist[k] = run;
                    run += c;
                }
            }
            __syncthreads();
            if (tid < nb) s_perm[s_hist[bucket] + pos] = tid;
            __syncthreads();
            // quantum: the round's sum of |a| spans 2^30 quanta.  A non-finite
            // amplitude has no quantum: the round's pixels become NaN below.
            const bool bad = !(suma <= 3.4028235e38f);
            const int ex = (suma > 0.f && !bad) ? ilogbf(suma) + 1 : 0;
            const float to_q = ldexpf(1.f, 30 - ex);
            if (tid < nb) {
                const int q = s_perm[tid];
                const float4 p0 = s_box[q][0], p1 = s_box[q][1];
                const int pk = __float_as_int(p1.w);
                const int bx0 = (pk & 0xff) - 1, bx1 = ((pk >> 8) & 0xff) - 1;
                const int by0 = ((pk >> 16) & 0xff) - 1, by1 = ((pk >> 24) & 0xff) - 1;
                const float amq = p0.w * to_q;
                const int w = bx1 - bx0 + 1, h = by1 - by0 + 1;
                const int hh = (w > 0 && h > 0) ? h : 0;
                const float dx0 = (float)bx0 - p0.x;
                float dy = (float)by0 - p0.y;
                int gr = by0 * T + bx0;
                for (int r = 0; r < hh; ++r) {
                    const float zy = fmaf(p1.z * dy, dy, p0.z), bxl = 2.f * p1.y * dy;
                    float dx = dx0;
                    int gi = gr;
                    for (int c = 0; c < w; ++c) {
                        const float v = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(p1.x, dx, bxl), zy)) - etau;
                        // branch-free: pixels outside the cut add an integer zero (measured
                        // faster than skipping them; the sums are the same)
                        atomicAdd(&s_iacc[gi], __float2int_rn(amq * fmaxf(v, 0.f)));
                        if (kCount) cnt += v > 0.f ? 1u : 0u;
                        dx += 1.f;
                        ++gi;
                    }
                    dy += 1.f;
                    gr += T;
                }
            }
            __syncthreads();
            const float from_q = ldexpf(1.f, ex - 30);
            for (int p = tid; p < T * T; p += NT) {
                const int v = s_iacc[p];
                if (bad) s_acc[p] = __builtin_nanf("");
                if (v != 0) {
                    if (!bad) s_acc[p] += (float)v * from_q;
                    s_iacc[p] = 0;
                }
            }
        }
        __syncthreads();
        float sq = 0.f;
        for (int p = tid; p < T * T; p += NT) {
            const int px = tc.x0 + p % T, py = tc.y0 + p / T;
            if (px < tc.W && py < tc.H) {
                const int64_t pi = tc.pix_off + (int64_t)py * tc.W + px;
                const float acc = s_acc[p];
                pred[pi] = acc;
                if (kLoss) {
                    const float m = mask[pi];
                    const float r = acc - target[pi];
                    loss_term(a.loss_kind, m, r, inv_msum, sq, grad ? grad + pi : nullptr);
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


// Epilogue of a tile whose sums are final: pred, and with kLoss the data
// term's gradient and the tile's loss partial tile_sse[tile].  acc holds the
// tile's T x T sums (tile-local row major).  Called by all threads of the
// workgroup; s_red holds a float per wave.
template <int T, int NT, bool kLoss>
__device__ inline void finish_tile(const RenderArgs& a, int tile, const float* acc, const TileOrg& o,
                                   const float* __restrict__ target, const float* __restrict__ mask,
                                   float inv_msum, float* __restrict__ pred, float* __restrict__ grad,
                                   float* __restrict__ tile_sse, float* s_red) {
    const int tid = threadIdx.x;
    float sq = 0.f;
    for (int p = tid; p < T * T; p += NT) {
        const int px = p % T, py = p / T;
        if (px < o.vw && py < o.vh) {
            const int64_t pi = o.base + (int64_t)py * o.stride + px;
            const float y = acc[p];
            pred[pi] = y;
            if (kLoss) loss_term(a.loss_kind, mask[pi], y - target[pi], inv_msum, sq, grad ? grad + pi : nullptr);
        }
    }
    if (kLoss) {
        for (int o2 = 32; o2 > 0; o2 >>= 1) sq += __shfl_xor(sq, o2, 64);
        if ((tid & 63) == 0) s_red[tid >> 6] = sq;
        __syncthreads();
        if (tid == 0) {
            float t = 0.f;
            for (int q = 0; q < NT / 64; ++q) t += s_red[q];
            tile_sse[tile] = t;
        }
        __syncthreads();
    }
}

// Forward, record per lane with exact integer accumulation, over fixed chunks
// of the tile-ordered instance list (the chunking of the adjoint): workgroup b
// takes instances [256 b, 256 b + 256), which may span a few tiles.  Per pass
// (up to KT of the chunk's tiles) the boxes are counting-sorted by shape in
// LDS (a wave's lanes then walk boxes of one shape), and each lane walks one
// box rows outer / columns inner and adds round(a max(e - e_T, 0) / quantum)
// to its tile's int32 LDS sum with an integer LDS atomic (float LDS atomics
// are slow on this GPU, integer ones are not).  The quantum is 2^(e - 30)
// with 2^e above the pass's sum of |a|, so no pixel's sum can overflow and
// the rounding error per term is below 2^-31 of that sum; integer sums do not
// depend on the order of the adds.  A tile whose instances all lie in the
// chunk is finished here; the first and the last tile of a chunk may run on
// into neighbouring chunks, and their sums go to the chunk's two partial
// slots, which k_forward_finish adds in chunk order.  The result is
// deterministic.
template <int T, bool kLoss, bool kCount>
__global__ __launch_bounds__(256) void k_forward_chunk(RenderArgs a, const float* __restrict__ target,
                                                       const float* __restrict__ mask,
                                                       const float* __restrict__ msum,
                                                       float* __restrict__ pred, float* __restrict__ grad,
                                                       float* __restrict__ tile_sse,
                                                       unsigned long long* __restrict__ incut,
                                                       float* __restrict__ partial) {
    constexpr int NT = 256, NW = 4;
    // shape buckets: box sides above 16 share the last bucket (a smaller
    // histogram to scan; measured faster at T = 32)
    constexpr int kS = T < 16 ? T : 16;
    constexpr int kB = (kS + 1) * (kS + 1);
    constexpr int KT = (1024 / (T * T)) > 0 ? 1024 / (T * T) : 1;
    __shared__ int s_iacc[KT * T * T];  // fixed-point sums, then (in place) their float values
    __shared__ float4 s_box[NT][2];
    __shared__ int s_gb[NT];
    __shared__ int s_hist[kB + 1];
    __shared__ int s_perm[NT];
    __shared__ int s_wsum[NW];
    __shared__ float s_fsum[NW];
    __shared__ float s_red[NW];
    __shared__ unsigned int s_cnt[NW];
    __shared__ int4 s_org[KT];  // the pass's tiles (TileOrg packing)
    __shared__ int s_ptile[KT];
    __shared__ int s_fin[KT];  // -1: tile finished here, else the partial slot (0 first run, 1 last run)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n_chunks = (a.n_inst + NT - 1) / NT;
    const int64_t chunk = xcd_tile(blockIdx.x, (int)n_chunks);
    if (chunk >= n_chunks) return;  // idle workgroup of the XCD remap (uniform)
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float* s_facc = reinterpret_cast<float*>(s_iacc);

    // every lane's instance: tile, run head, record and box (independent loads)
    const int64_t inst = chunk * NT + tid;
    int tile = -1;
    bool head = false;
    int4 org = make_int4(0, 0, 0, 0);
    if (inst < a.n_inst) {
        const uint32_t t = a.inst_key[inst] >> kClassBits;
        if (t < (uint32_t)a.n_tiles) {
            tile = (int)t;
            head = tid == 0 || (a.inst_key[inst - 1] >> kClassBits) != t;
            org = a.tile_org[tile];
        }
    }
    for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
    const uint64_t hm = __ballot(head);
    if (lane == 0) s_wsum[wv] = __popcll(hm);
    int bucket = 0;
    float absa = 0.f;
    int fin = -1;
    if (tile >= 0) {
        const Record R = a.rec[a.inst_rec[inst]];
        const TileOrg o = tile_org(org);
        const LaneBox b = lane_box(R, o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
        const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
        const bool empty = w == 0 || h == 0;
        const int x0 = empty ? 0 : b.x0, x1 = empty ? -1 : b.x1;
        const int y0 = empty ? 0 : b.y0, y1 = empty ? -1 : b.y1;
        bucket = empty ? 0 : (min(h, kS) * (kS + 1) + min(w, kS));
        absa = empty ? 0.f : fabsf(b.am);
        s_box[tid][0] = make_float4(b.pxl, b.pyl, b.bz, b.am);
        s_box[tid][1] = make_float4(b.a00, b.a01, b.a11,
                                    __int_as_float((x0 + 1) | ((x1 + 1) << 8) | ((y0 + 1) << 16) |
                                                   ((y1 + 1) << 24)));
        if (head) {
            const int2 rg = a.ranges[tile];
            const bool inside = rg.x >= chunk * NT && rg.y <= chunk * NT + NT;
            fin = inside ? -1 : (tid == 0 ? 0 : 1);
        }
    }
    __syncthreads();
    int rslot = __popcll(hm & ((1ull << lane) - 1ull)) + (head ? 1 : 0) - 1;
    int nd = 0;
    for (int q = 0; q < NW; ++q) {
        if (q < wv) rslot += s_wsum[q];
        nd += s_wsum[q];
    }
    unsigned int cnt = 0;
    for (int p0 = 0; p0 < nd; p0 += KT) {
        const int np = min(KT, nd - p0);
        if (p0 > 0) {
            __syncthreads();  // the previous pass is done with LDS
            for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
        }
        const bool act = tile >= 0 && rslot >= p0 && rslot < p0 + np;
        if (act && head) {
            s_org[rslot - p0] = org;
            s_ptile[rslot - p0] = tile;
            s_fin[rslot - p0] = fin;
        }
        for (int q = tid; q < np * T * T; q += NT) s_iacc[q] = 0;
        // the pass's sum of |a| (its instances only)
        float pa = act ? absa : 0.f;
        for (int o = 32; o > 0; o >>= 1) pa += __shfl_xor(pa, o, 64);
        if (lane == 0) s_fsum[wv] = pa;
        __syncthreads();
        int pos = 0;
        if (act) {
            s_gb[tid] = (rslot - p0) * T * T;
            pos = atomicAdd(&s_hist[bucket], 1);
        }
        const float suma = (s_fsum[0] + s_fsum[1]) + (s_fsum[2] + s_fsum[3]);
        __syncthreads();
        {   // exclusive scan of the bucket counts; s_hist[kB] receives the total
            const int per = (kB + NT - 1) / NT;
            const int kb = min(tid * per, kB), ke = min(kb + per, kB);
            int local = 0;
            for (int k = kb; k < ke; ++k) local += s_hist[k];
            int incl = local;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o) incl += u;
            }
            if (lane == 63) s_wsum[wv] = incl;
            __syncthreads();
            int run = incl - local;
            for (int q = 0; q < wv; ++q) run += s_wsum[q];
            for (int k = kb; k < ke; ++k) {
                const int c = s_hist[k];
                s_hist[k] = run;
                run += c;
            }
            if (kb < kB && ke == kB) s_hist[kB] = run;
        }
        __syncthreads();
        if (act) s_perm[s_hist[bucket] + pos] = tid;
        __syncthreads();
        // quantum: the pass's sum of |a| spans 2^30 quanta.  A non-finite
        // amplitude has no quantum: the pass's pixels become NaN below.
        const bool bad = !(suma <= 3.4028235e38f);
        const int ex = (suma > 0.f && !bad) ? ilogbf(suma) + 1 : 0;
        const float to_q = ldexpf(1.f, 30 - ex);
        if (tid < s_hist[kB]) {
            const int q = s_perm[tid];
            const float4 p0v = s_box[q][0], p1 = s_box[q][1];
            const int pk = __float_as_int(p1.w);
            const int bx0 = (pk & 0xff) - 1, bx1 = ((pk >> 8) & 0xff) - 1;
            const int by0 = ((pk >> 16) & 0xff) - 1, by1 = ((pk >> 24) & 0xff) - 1;
            const float amq = p0v.w * to_q;
            const int w = bx1 - bx0 + 1, h = by1 - by0 + 1;
            const int hh = (w > 0 && h > 0) ? h : 0;
            const float dx0 = (float)bx0 - p0v.x;
            float dy = (float)by0 - p0v.y;
            int gr = s_gb[q] + by0 * T + bx0;
            for (int r = 0; r < hh; ++r) {
                const float zy = fmaf(p1.z * dy, dy, p0v.z), bxl = 2.f * p1.y * dy;
                float dx = dx0;
                int gi = gr;
                for (int c = 0; c < w; ++c) {
                    const float v = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(p1.x, dx, bxl), zy)) - etau;
                    // branch-free: pixels outside the cut add an integer zero (measured
                    // faster than skipping them; the sums are the same)
                    atomicAdd(&s_iacc[gi], __float2int_rn(amq * fmaxf(v, 0.f)));
                    if (kCount) cnt += v > 0.f ? 1u : 0u;
                    dx += 1.f;
                    ++gi;
                }
                dy += 1.f;
                gr += T;
            }
        }
        __syncthreads();
        const float from_q = ldexpf(1.f, ex - 30);
        for (int q = tid; q < np * T * T; q += NT) s_facc[q] = bad ? __builtin_nanf("") : (float)s_iacc[q] * from_q;
        __syncthreads();
        for (int sl = 0; sl < np; ++sl) {
            const int f = s_fin[sl];
            if (f < 0) {
                const TileOrg o = tile_org(s_org[sl]);
                finish_tile<T, NT, kLoss>(a, s_ptile[sl], s_facc + sl * T * T, o, target, mask, inv_msum, pred,
                                          grad, tile_sse, s_red);
            } else {
                float* dst = partial + ((size_t)chunk * 2 + f) * (T * T);
                for (int p = tid; p < T * T; p += NT) dst[p] = s_facc[sl * T * T + p];
            }
        }
    }
    if (kCount) {
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) s_cnt[wv] = cnt;
        __syncthreads();
        if (tid == 0) {
            unsigned long long c = 0;
            for (int q = 0; q < NW; ++q) c += s_cnt[q];
            if (c) atomicAdd(incut, c);
        }
    }
}

// Tiles that k_forward_chunk did not finish: those without instances (sums
// zero) and those whose instances span several chunks (sums = the chunks'
// partial slots added in chunk order: the tile is the last run of its first
// chunk unless it starts that chunk, and the first run of every later one).
template <int T, bool kLoss>
__global__ __launch_bounds__(256) void k_forward_finish(RenderArgs a, const float* __restrict__ target,
                                                        const float* __restrict__ mask,
                                                        const float* __restrict__ msum,
                                                        float* __restrict__ pred, float* __restrict__ grad,
                                                        float* __restrict__ tile_sse,
                                                        const float* __restrict__ partial) {
    constexpr int NT = 256;
    __shared__ float s_acc[T * T];
    __shared__ float s_red[NT / 64];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    const int2 rg = a.ranges[tile];
    const int64_t c0 = rg.y > rg.x ? rg.x / NT : 0, c1 = rg.y > rg.x ? (rg.y - 1) / NT : -1;
    if (rg.y > rg.x && c0 == c1) return;  // finished by its chunk
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    // every thread's pixels, summed over the chunks in chunk order; the loads
    // of eight chunks are issued together (a tile spans tens of chunks)
    constexpr int PPT = (T * T + NT - 1) / NT;
    constexpr int U = 8;
    float acc[PPT];
    for (int k = 0; k < PPT; ++k) acc[k] = 0.f;
    for (int64_t cb = c0; cb <= c1; cb += U) {
        float v[U][PPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = cb + u;
            const int ps = (c == c0 && rg.x != c0 * NT) ? 1 : 0;
            const float* src = partial + ((size_t)c * 2 + ps) * (T * T);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int p = threadIdx.x + k * NT;
                v[u][k] = (c <= c1 && p < T * T) ? src[p] : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < PPT; ++k) acc[k] += v[u][k];
    }
    for (int k = 0; k < PPT; ++k) {
        const int p = threadIdx.x + k * NT;
        if (p < T * T) s_acc[p] = acc[k];
    }
    finish_tile<T, NT, kLoss>(a, tile, s_acc, tile_org(a.tile_org[tile]), target, mask, inv_msum, pred, grad,
                              tile_sse, s_red);
}

// Forward, record on lanes: a batch of the tile's records is staged in LDS
// (footprint box, 1/width and the exponent as a quadratic in box-local pixel
// coordinates).  Each group of 16 lanes (one DPP row) then takes one instance
// at a time, spreads the instance's box over its lanes (16 pixels per pass:
// pixel k of the box is row floor((k + 1/2) / w), which a float reciprocal
// gets exactly for boxes of at most 32 x 32) and adds
// a * max(e - e_T, 0) into its own LDS copy of the tile with a plain
// read-modify-write (measured faster here than LDS float atomics): the lanes
// of one group hit distinct pixels and no other group touches that copy.
// The sixteen copies are then summed in a fixed order, so the result needs
// no atomics and is deterministic.  Footprints are small (tens of pixels),
// so 16-lane groups waste fewer lanes on a box's last pass than half-waves
// and spread the per-instance set-up over four instances per instruction.
// Instances are grouped by footprint size in the sort, so the four groups of
// a wave see similar boxes.
template <int T, bool kLoss, bool kCount>
__global__ __launch_bounds__(256) void k_forward_rol(RenderArgs a, const float* __restrict__ target,
                                                     const float* __restrict__ mask,
                                                     const float* __restrict__ msum,
                                                     float* __restrict__ pred, float* __restrict__ grad,
                                                     float* __restrict__ tile_sse,
                                                     unsigned long long* __restrict__ incut,
                                                     int* __restrict__ work_counter) {
    constexpr int NT = 256, NW = 4, NG = 16, NH = NT / NG;
    constexpr int kCopy = T * T + 8;  // copy stride: successive copies start 8 banks apart
    __shared__ float s_acc[NH * kCopy];
    __shared__ float4 s_rec[kMaxBatch][3];
    __shared__ float s_red[NW];
    __shared__ unsigned int s_cnt[NW];
    __shared__ int s_next;
    const int tid = threadIdx.x, lane = tid & 63, hl = tid & (NG - 1);
    const int wv = tid >> 6, grp = tid / NG;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float* acc = s_acc + grp * kCopy;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile < 0) break;
        const TileCoord tc = tile_coord(a, tile);
        const int2 rg = a.ranges[tile];
        const int xmax = min(T, tc.W - tc.x0) - 1, ymax = min(T, tc.H - tc.y0) - 1;
        __syncthreads();
        for (int p = tid; p < NH * kCopy; p += NT) s_acc[p] = 0.f;
        unsigned int cnt = 0;
        for (int b0 = rg.x; b0 < rg.y; b0 += a.batch) {
            const int nb = min(a.batch, rg.y - b0);
            __syncthreads();
            for (int q = tid; q < nb; q += NT) {
                const Record R = a.rec[a.inst_rec[b0 + q]];
                const LaneBox b = lane_box(R, tc.x0, tc.y0, xmax, ymax, tau2k);
                const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
                // exponent at box-local (u, v) = (x - x0, y - y0): expand around the box origin
                const float PX = b.pxl - (float)b.x0, PY = b.pyl - (float)b.y0;
                float4 c0, c1, c2;
                c0.x = b.bz + PX * (b.a00 * PX + 2.f * b.a01 * PY) + b.a11 * PY * PY;
                c0.y = -2.f * (b.a00 * PX + b.a01 * PY);
                c0.z = -2.f * (b.a01 * PX + b.a11 * PY);
                c0.w = b.a00;
                c1.x = 2.f * b.a01;
                c1.y = b.a11;
                c1.z = b.am;
                c1.w = __int_as_float(w * h);
                const float rw = __builtin_amdgcn_rcpf((float)max(w, 1));
                c2.x = rw;
                c2.y = 0.5f * rw;
                c2.z = (float)w;
                c2.w = __int_as_float(b.y0 * T + b.x0);  // offset of the box origin in a copy
                s_rec[q][0] = c0;
                s_rec[q][1] = c1;
                s_rec[q][2] = c2;
            }
            __syncthreads();
            for (int q = grp; q < nb; q += NH) {
                const float4 c0 = s_rec[q][0], c1 = s_rec[q][1], c2 = s_rec[q][2];
                const int area = __float_as_int(c1.w);
                // small integers are exact in float: pixel k of the box sits at
                // row v = trunc((k + 1/2) / w), column u = k - v w, and at
                // offset org + k + v (T - w) in the copy
                const float farea = (float)area, fskip = (float)T - c2.z;
                const float base = (float)__float_as_int(c2.w) + (float)hl;
                __builtin_amdgcn_s_waitcnt(0xc07f);  // staged values in registers before the pixel loop
                for (int c = 0; c < area; c += NG) {
                    const float fk = (float)(c + hl);
                    const float v = truncf(fmaf(fk, c2.x, c2.y));
                    const float u = fmaf(-v, c2.z, fk);
                    float z = fmaf(c0.w, u, fmaf(c1.x, v, c0.y));
                    z = fmaf(z, u, c0.x);
                    z = fmaf(fmaf(c1.y, v, c0.z), v, z);
                    const float e = __builtin_amdgcn_exp2f(z) - etau;
                    if (fk < farea && e > 0.f) {
                        float* dst = acc + (int)fmaf(v, fskip, base + (float)c);
                        *dst = fmaf(c1.z, e, *dst);
                        if (kCount) ++cnt;
                    }
                }
            }
        }
        __syncthreads();
        float sq = 0.f;
        for (int p = tid; p < T * T; p += NT) {
            const int px = tc.x0 + p % T, py = tc.y0 + p / T;
            if (px < tc.W && py < tc.H) {
                const int64_t pi = tc.pix_off + (int64_t)py * tc.W + px;
                const float* r = s_acc + p;
                float part[NH / 2];
                for (int q = 0; q < NH / 2; ++q) part[q] = r[(2 * q) * kCopy] + r[(2 * q + 1) * kCopy];
                for (int h = NH / 4; h > 0; h >>= 1)
                    for (int q = 0; q < h; ++q) part[q] = part[2 * q] + part[2 * q + 1];
                const float y = part[0];
                pred[pi] = y;
                if (kLoss) {
                    const float m = mask[pi];
                    const float rr = y - target[pi];
                    loss_term(a.loss_kind, m, rr, inv_msum, sq, grad ? grad + pi : nullptr);
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
                unsigned long long cc = 0;
                for (int q = 0; q < NW; ++q) {
                    t += s_red[q];
                    cc += s_cnt[q];
                }
                if (kLoss) tile_sse[tile] = t;
                if (kCount && cc) atomicAdd(incut, cc);
            }
        }
    }
}

// Adjoint, record per lane, persistent grid (persistent = 1): workgroups pull
// whole tiles heaviest-first from a work queue; the tile's upstream gradient
// is staged in LDS and every lane walks one instance's box and sums, with
// t = g e (inside the cut):
//   Sa = sum g max(e - e_T, 0), S0 = sum t, Sx = sum t dx, Sy = sum t dy,
//   Sxx = sum t dx^2, Sxy = sum t dx dy, Syy = sum t dy^2,
// from which the gradient with respect to the stored record fields follows
// (dz/d field, times amp ln 2).  The result goes to the instance's emission
// slot, so no atomics are needed.  The walk is rows outer, columns inner,
// with per-row sums folded in with dy (three accumulations per pixel instead
// of seven).  A wave runs each loop as long as its largest trip count, so
// each round of up to 256 instances is first ordered by (box height, box
// width) with a counting sort in LDS, and lane j walks the j-th box: the
// lanes of a wave then have boxes of the same shape.  Which lane walks which
// instance changes no instance's sum, so the result stays deterministic.
template <int T, int NT>
__global__ __launch_bounds__(NT) void k_backward_tiles(RenderArgs a, const float* __restrict__ grad_pred,
                                                 const float* __restrict__ grad_scale,
                                                 float4* __restrict__ inst_grad,
                                                 int* __restrict__ work_counter) {
    constexpr int kB = (T + 1) * (T + 1);
    __shared__ float s_g[T * T];
    __shared__ float4 s_box[NT][2];
    __shared__ uint32_t s_slot[NT];
    __shared__ int s_hist[kB + 1];
    __shared__ int s_perm[NT];
    __shared__ int s_wsum[NT / 64];
    __shared__ int s_next;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float scale = grad_scale ? grad_scale[0] : 1.f;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile < 0) break;
        const TileCoord tc = tile_coord(a, tile);
        const int2 rg = a.ranges[tile];
        const int xmax = min(T, tc.W - tc.x0) - 1, ymax = min(T, tc.H - tc.y0) - 1;
        __syncthreads();
        for (int p = tid; p < T * T; p += NT) {
            const int px = tc.x0 + p % T, py = tc.y0 + p / T;
            s_g[p] = (px < tc.W && py < tc.H) ? grad_pred[tc.pix_off + (int64_t)py * tc.W + px] * scale : 0.f;
        }
        const int n = rg.y - rg.x;
        for (int r0 = 0; r0 < n; r0 += NT) {
            const int cnt = min(NT, n - r0);
            __syncthreads();
            for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
            __syncthreads();
            int bucket = 0, pos = 0;
            if (tid < cnt) {
                const Record R = a.rec[a.inst_rec[rg.x + r0 + tid]];
                const LaneBox b = lane_box(R, tc.x0, tc.y0, xmax, ymax, tau2k);
                const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
                const bool empty = w == 0 || h == 0;
                const int x0 = empty ? 0 : b.x0, x1 = empty ? -1 : b.x1;
                const int y0 = empty ? 0 : b.y0, y1 = empty ? -1 : b.y1;
                bucket = empty ? 0 : (h * (T + 1) + w);
                s_box[tid][0] = make_float4(b.pxl, b.pyl, b.bz, b.am);
                s_box[tid][1] = make_float4(b.a00, b.a01, b.a11,
                                            __int_as_float((x0 + 1) | ((x1 + 1) << 8) | ((y0 + 1) << 16) |
                                                           ((y1 + 1) << 24)));
                s_slot[tid] = a.inst_idx[rg.x + r0 + tid];
                pos = atomicAdd(&s_hist[bucket], 1);
            }
            __syncthreads();
            {   // exclusive scan of the bucket counts: thread t takes a run of ceil(kB / NT)
                const int per = (kB + NT - 1) / NT;
                const int kb = min(tid * per, kB), ke = min(kb + per, kB);
                int local = 0;
                for (int k = kb; k < ke; ++k) local += s_hist[k];
                int incl = local;
                for (int o = 1; o < 64; o <<= 1) {
                    const int u = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += u;
                }
                if (lane == 63) s_wsum[wv] = incl;
                __syncthreads();
                int run = incl - local;
                for (int q = 0; q < wv; ++q) run += s_wsum[q];
                for (int k = kb; k < ke; ++k) {
                    const int c = s_hist[k];
                    s_hist[k] = run;
                    run += c;
                }
            }
            __syncthreads();
            if (tid < cnt) s_perm[s_hist[bucket] + pos] = tid;
            __syncthreads();
            if (tid < cnt) {
                const int q = s_perm[tid];
                const float4 p0 = s_box[q][0], p1 = s_box[q][1];
                const int pk = __float_as_int(p1.w);
                const int bx0 = (pk & 0xff) - 1, bx1 = ((pk >> 8) & 0xff) - 1;
                const int by0 = ((pk >> 16) & 0xff) - 1, by1 = ((pk >> 24) & 0xff) - 1;
                const float pxl = p0.x, pyl = p0.y, bz = p0.z, am = p0.w;
                const float a00 = p1.x, a01 = p1.y, a11 = p1.z;
                float S0 = 0.f, Sx = 0.f, Sy = 0.f, Sxx = 0.f, Sxy = 0.f, Syy = 0.f, Sa = 0.f;
                const int w = bx1 - bx0 + 1, h = by1 - by0 + 1;
                const int hh = (w > 0 && h > 0) ? h : 0;
                const float dx0 = (float)bx0 - pxl;
                const float b2a01 = 2.f * a01;
                float dy = (float)by0 - pyl;
                int gr = by0 * T + bx0;
                for (int r = 0; r < hh; ++r) {
                    const float zy = fmaf(a11 * dy, dy, bz), bxl = b2a01 * dy;
                    float R0 = 0.f, R1 = 0.f, R2 = 0.f, dx = dx0;
                    int gi = gr;
                    for (int c = 0; c < w; ++c) {
                        const float g = s_g[gi];
                        const float e = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(a00, dx, bxl), zy));
                        const float v = e - etau;
                        Sa = fmaf(g, fmaxf(v, 0.f), Sa);
                        const float t = (v > 0.f) ? g * e : 0.f;
                        const float tx = t * dx;
                        R0 += t;
                        R1 += tx;
                        R2 = fmaf(tx, dx, R2);
                        dx += 1.f;
                        ++gi;
                    }
                    S0 += R0;
                    Sx += R1;
                    Sxx += R2;
                    Sy = fmaf(dy, R0, Sy);
                    Sxy = fmaf(dy, R1, Sxy);
                    Syy = fmaf(dy * dy, R0, Syy);
                    dy += 1.f;
                    gr += T;
                }
                const float k2 = am * SVR_LN2;
                float4 g0, g1;
                g0.x = Sa;
                g0.y = k2 * S0;
                g0.z = -2.f * k2 * (a00 * Sx + a01 * Sy);
                g0.w = -2.f * k2 * (a01 * Sx + a11 * Sy);
                g1.x = k2 * Sxx;
                g1.y = 2.f * k2 * Sxy;
                g1.z = k2 * Syy;
                g1.w = 0.f;
                const uint32_t e_slot = s_slot[q];
                inst_grad[2 * (int64_t)e_slot] = g0;
                inst_grad[2 * (int64_t)e_slot + 1] = g1;
            }
        }
    }
}


// Adjoint, record per lane, over fixed chunks of the sorted instance list:
// workgroup b takes instances [256 b, 256 b + 256), which are ordered by tile
// and may span several tiles, so every workgroup has one full round of work
// whatever the instance count of a tile, and the grid load stays even (one
// workgroup per tile left the chip with a long tail of busy tiles).  The
// upstream gradients of the chunk's tiles are staged in LDS (up to KT tiles at
// a time; a chunk over more tiles takes further passes); every lane walks one
// instance's box and sums, with t = g e (inside the cut):
//   Sa = sum g max(e - e_T, 0), S0 = sum t, Sx = sum t dx, Sy = sum t dy,
//   Sxx = sum t dx^2, Sxy = sum t dx dy, Syy = sum t dy^2,
// from which the gradient with respect to the stored record fields follows
// (dz/d field, times amp ln 2).  The result goes to the instance's emission
// slot, so no atomics are needed.  The walk is rows outer, columns inner,
// with per-row sums folded in with dy (three accumulations per pixel instead
// of seven).  A wave runs each loop as long as its largest trip count, so the
// pass's instances are first ordered by (box height, box width) with a
// counting sort in LDS, and lane j walks the j-th box: the lanes of a wave
// then have boxes of the same shape.  Which lane walks which instance changes
// no instance's sum, so the result is deterministic and independent of the
// chunking.
template <int T, int NT>
__global__ __launch_bounds__(NT) void k_backward(RenderArgs a, const float* __restrict__ grad_pred,
                                                 const float* __restrict__ grad_scale,
                                                 float4* __restrict__ inst_grad) {
    constexpr int kB = (T + 1) * (T + 1);
    constexpr int KT = (1024 / (T * T)) > 0 ? 1024 / (T * T) : 1;  // tiles staged per pass (4 KB)
    constexpr int NW = NT / 64;
    __shared__ float s_g[KT * T * T];
    __shared__ float4 s_box[NT][2];
    __shared__ uint32_t s_slot[NT];
    __shared__ int s_gb[NT];
    __shared__ int s_hist[kB + 1];
    __shared__ int s_perm[NT];
    __shared__ int s_wsum[NW];
    __shared__ int4 s_org[KT];  // the pass's tiles (TileOrg packing)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n_chunks = (a.n_inst + NT - 1) / NT;
    const int64_t chunk = xcd_tile(blockIdx.x, (int)n_chunks);
    if (chunk >= n_chunks) return;  // idle workgroup of the XCD remap (uniform)
    const float tau2k = SVR_KZ * a.tau2;
    const float etau = a.etau;

    // every lane's instance: tile (-1 past the end or for emission padding),
    // whether it heads a run of its tile in the chunk, its record and box;
    // the loads are independent so their latencies overlap
    const int64_t inst = chunk * NT + tid;
    int tile = -1;
    bool head = false;
    int4 org = make_int4(0, 0, 0, 0);
    if (inst < a.n_inst) {
        const uint32_t t = a.inst_key[inst] >> kClassBits;
        if (t < (uint32_t)a.n_tiles) {
            tile = (int)t;
            head = tid == 0 || (a.inst_key[inst - 1] >> kClassBits) != t;
            org = a.tile_org[tile];
        }
    }
    for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
    const uint64_t hm = __ballot(head);
    if (lane == 0) s_wsum[wv] = __popcll(hm);
    int bucket = 0;
    if (tile >= 0) {
        const Record R = a.rec[a.inst_rec[inst]];
        const TileOrg o = tile_org(org);
        const LaneBox b = lane_box(R, o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
        const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
        const bool empty = w == 0 || h == 0;
        const int bx0 = empty ? 0 : b.x0, bx1 = empty ? -1 : b.x1;
        const int by0 = empty ? 0 : b.y0, by1 = empty ? -1 : b.y1;
        bucket = empty ? 0 : (h * (T + 1) + w);
        s_box[tid][0] = make_float4(b.pxl, b.pyl, b.bz, b.am);
        s_box[tid][1] = make_float4(b.a00, b.a01, b.a11,
                                    __int_as_float((bx0 + 1) | ((bx1 + 1) << 8) | ((by0 + 1) << 16) |
                                                   ((by1 + 1) << 24)));
        s_slot[tid] = a.inst_idx[inst];
    }
    __syncthreads();
    // rslot = index of the lane's run (distinct tile) in the chunk
    int rslot = __popcll(hm & ((1ull << lane) - 1ull)) + (head ? 1 : 0) - 1;
    int nd = 0;
    for (int q = 0; q < NW; ++q) {
        if (q < wv) rslot += s_wsum[q];
        nd += s_wsum[q];
    }
    for (int p0 = 0; p0 < nd; p0 += KT) {
        const int np = min(KT, nd - p0);
        if (p0 > 0) {
            __syncthreads();  // the previous pass is done with LDS
            for (int k = tid; k < kB; k += NT) s_hist[k] = 0;
        }
        const bool act = tile >= 0 && rslot >= p0 && rslot < p0 + np;
        if (act && head) s_org[rslot - p0] = org;
        __syncthreads();  // s_org and the zeroed histogram are visible
        int pos = 0;
        if (act) {
            s_gb[tid] = (rslot - p0) * T * T;
            pos = atomicAdd(&s_hist[bucket], 1);
        }
        for (int q = tid; q < np * T * T; q += NT) {
            const int sl = q / (T * T), pix = q - sl * (T * T);
            const TileOrg o = tile_org(s_org[sl]);
            const int px = pix % T, py = pix / T;
            float gv = 0.f;
            if (px < o.vw && py < o.vh) gv = grad_pred[o.base + (int64_t)py * o.stride + px];
            s_g[q] = gv;
        }
        __syncthreads();
        {   // exclusive scan of the bucket counts: thread t takes a run of
            // ceil(kB / NT); s_hist[kB] receives the total
            const int per = (kB + NT - 1) / NT;
            const int kb = min(tid * per, kB), ke = min(kb + per, kB);
            int local = 0;
            for (int k = kb; k < ke; ++k) local += s_hist[k];
            int incl = local;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o) incl += u;
            }
            if (lane == 63) s_wsum[wv] = incl;
            __syncthreads();
            int acc = incl - local;
            for (int q = 0; q < wv; ++q) acc += s_wsum[q];
            for (int k = kb; k < ke; ++k) {
                const int c = s_hist[k];
                s_hist[k] = acc;
                acc += c;
            }
            if (kb < kB && ke == kB) s_hist[kB] = acc;
        }
        __syncthreads();
        if (act) s_perm[s_hist[bucket] + pos] = tid;
        __syncthreads();
        const float scale = grad_scale ? grad_scale[0] : 1.f;
        if (tid < s_hist[kB]) {
            const int q = s_perm[tid];
            const float4 p0v = s_box[q][0], p1 = s_box[q][1];
            const int pk = __float_as_int(p1.w);
            const int bx0 = (pk & 0xff) - 1, bx1 = ((pk >> 8) & 0xff) - 1;
            const int by0 = ((pk >> 16) & 0xff) - 1, by1 = ((pk >> 24) & 0xff) - 1;
            const float pxl = p0v.x, pyl = p0v.y, bz = p0v.z, am = p0v.w;
            const float a00 = p1.x, a01 = p1.y, a11 = p1.z;
            float S0 = 0.f, Sx = 0.f, Sy = 0.f, Sxx = 0.f, Sxy = 0.f, Syy = 0.f, Sa = 0.f;
            const int w = bx1 - bx0 + 1, h = by1 - by0 + 1;
            const int hh = (w > 0 && h > 0) ? h : 0;
            const float dx0 = (float)bx0 - pxl;
            const float b2a01 = 2.f * a01;
            float dy = (float)by0 - pyl;
            int gr = s_gb[q] + by0 * T + bx0;
            for (int r = 0; r < hh; ++r) {
                const float zy = fmaf(a11 * dy, dy, bz), bxl = b2a01 * dy;
                float R0 = 0.f, R1 = 0.f, R2 = 0.f, dx = dx0;
                int gi = gr;
                for (int c = 0; c < w; ++c) {
                    const float g = s_g[gi];
                    const float e = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(a00, dx, bxl), zy));
                    const float v = e - etau;
                    Sa = fmaf(g, fmaxf(v, 0.f), Sa);
                    const float t = (v > 0.f) ? g * e : 0.f;
                    const float tx = t * dx;
                    R0 += t;
                    R1 += tx;
                    R2 = fmaf(tx, dx, R2);
                    dx += 1.f;
                    ++gi;
                }
                S0 += R0;
                Sx += R1;
                Sxx += R2;
                Sy = fmaf(dy, R0, Sy);
                Sxy = fmaf(dy, R1, Sxy);
                Syy = fmaf(dy * dy, R0, Syy);
                dy += 1.f;
                gr += T;
            }
            // the upstream scale multiplies every sum (it was applied to g)
            const float k2 = am * SVR_LN2 * scale;
            float4 g0, g1;
            g0.x = Sa * scale;
            g0.y = k2 * S0;
            g0.z = -2.f * k2 * (a00 * Sx + a01 * Sy);
            g0.w = -2.f * k2 * (a01 * Sx + a11 * Sy);
            g1.x = k2 * Sxx;
            g1.y = 2.f * k2 * Sxy;
            g1.z = k2 * Syy;
            g1.w = 0.f;
            const uint32_t e_slot = s_slot[q];
            inst_grad[2 * (int64_t)e_slot] = g0;
            inst_grad[2 * (int64_t)e_slot + 1] = g1;
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
        const int per_cu = threads >= 256 ? 8 : (threads >= 128 ? 16 : 32);
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

template <int T>
hipError_t fwd_rol_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                            float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                            int* work_counter, int grid, hipStream_t st) {
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    if (loss && count)
        hipLaunchKernelGGL((k_forward_rol<T, true, true>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else if (loss)
        hipLaunchKernelGGL((k_forward_rol<T, true, false>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else if (count)
        hipLaunchKernelGGL((k_forward_rol<T, false, true>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else
        hipLaunchKernelGGL((k_forward_rol<T, false, false>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    return hipGetLastError();
}

template <int T>
hipError_t fwd_rpl_tiles_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                                  float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                                  int* work_counter, int grid, hipStream_t st) {
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    if (loss && count)
        hipLaunchKernelGGL((k_forward_rpl_tiles<T, true, true>), dim3(grid), dim3(256), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else if (loss)
        hipLaunchKernelGGL((k_forward_rpl_tiles<T, true, false>), dim3(grid), dim3(256), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else if (count)
        hipLaunchKernelGGL((k_forward_rpl_tiles<T, false, true>), dim3(grid), dim3(256), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    else
        hipLaunchKernelGGL((k_forward_rpl_tiles<T, false, false>), dim3(grid), dim3(256), 0, st, a, target, mask,
                           msum, pred, grad, tile_sse, incut, work_counter);
    return hipGetLastError();
}

template <int T>
hipError_t fwd_chunk_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                              float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                              float* partial, hipStream_t st) {
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    constexpr int NT = 256;
    const int64_t n_chunks = (a.n_inst + NT - 1) / NT;
    if (n_chunks > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    if (n_chunks > 0) {
        if (!partial) return hipErrorInvalidValue;
        const int grid = (int)(((n_chunks + 7) >> 3) << 3);  // whole XCD remap
        if (loss && count)
            hipLaunchKernelGGL((k_forward_chunk<T, true, true>), dim3(grid), dim3(NT), 0, st, a, target, mask, msum,
                               pred, grad, tile_sse, incut, partial);
        else if (loss)
            hipLaunchKernelGGL((k_forward_chunk<T, true, false>), dim3(grid), dim3(NT), 0, st, a, target, mask, msum,
                               pred, grad, tile_sse, incut, partial);
        else if (count)
            hipLaunchKernelGGL((k_forward_chunk<T, false, true>), dim3(grid), dim3(NT), 0, st, a, target, mask, msum,
                               pred, grad, tile_sse, incut, partial);
        else
            hipLaunchKernelGGL((k_forward_chunk<T, false, false>), dim3(grid), dim3(NT), 0, st, a, target, mask, msum,
                               pred, grad, tile_sse, incut, partial);
    }
    const int tgrid = ((a.n_tiles + 7) >> 3) << 3;
    if (loss)
        hipLaunchKernelGGL((k_forward_finish<T, true>), dim3(tgrid), dim3(NT), 0, st, a, target, mask, msum, pred,
                           grad, tile_sse, (const float*)partial);
    else
        hipLaunchKernelGGL((k_forward_finish<T, false>), dim3(tgrid), dim3(NT), 0, st, a, target, mask, msum, pred,
                           grad, tile_sse, (const float*)partial);
    return hipGetLastError();
}

size_t forward_partial_floats(const RenderArgs& a) {
    if (a.forward_mode != 1 || a.persistent || a.n_inst <= 0) return 0;
    const int64_t n_chunks = (a.n_inst + 255) / 256;
    return (size_t)n_chunks * 2 * (size_t)a.tile * (size_t)a.tile;
}

hipError_t launch_forward(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                          float* pred, float* grad_pred, float* tile_sse, unsigned long long* incut,
                          int* work_counter, float* partial, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (a.persistent) {
        hipError_t e = launch_fill_zero(work_counter, sizeof(int), st);
        if (e != hipSuccess) return e;
    }
    if (a.forward_mode == 2) {
        const int grid = grid_for(a, 256);
        switch (a.tile) {
            case 8: return fwd_rol_dispatch<8>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 16: return fwd_rol_dispatch<16>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 32: return fwd_rol_dispatch<32>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.forward_mode == 1 && a.persistent) {
        const int grid = grid_for(a, 256);
        switch (a.tile) {
            case 8: return fwd_rpl_tiles_dispatch<8>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 16: return fwd_rpl_tiles_dispatch<16>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 32: return fwd_rpl_tiles_dispatch<32>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.forward_mode == 1) {
        switch (a.tile) {
            case 8: return fwd_chunk_dispatch<8>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            case 16: return fwd_chunk_dispatch<16>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            case 32: return fwd_chunk_dispatch<32>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.tile) {
        case 8: return fwd_dispatch<8, 1>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 64), st);
        case 16: return fwd_dispatch<16, 1>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 256), st);
        case 32: return fwd_dispatch<32, 4>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid_for(a, 256), st);
        default: return hipErrorInvalidValue;
    }
}

// Scale regulariser of Eq. 7 on s = exp(log s): g += 2 lambda (s - s_t) s per
// log-scale, and the block's share of lambda sum (s - s_t)^2 into partial[].
__global__ __launch_bounds__(256) void k_scale_reg(const float* __restrict__ log_scale, int64_t n3, float lambda,
                                                   float s_target, float* __restrict__ g,
                                                   float* __restrict__ partial) {
    __shared__ float s[4];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
        const float sc = expf(log_scale[i]);
        const float d = sc - s_target;
        g[i] += 2.f * lambda * d * sc;
        acc = fmaf(d, d, acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = lambda * (s[0] + s[1] + s[2] + s[3]);
}

__global__ void k_add_sum(const float* __restrict__ partial, int n, float* __restrict__ out) {
    __shared__ float s[4];
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] += s[0] + s[1] + s[2] + s[3];
}

hipError_t launch_scale_reg(const float* log_scale, int64_t n, float lambda, float s_target, float* g, float* loss,
                            float* partial, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nb = kRegBlocks;
    hipLaunchKernelGGL(k_scale_reg, dim3(nb), dim3(256), 0, st, log_scale, 3 * n, lambda, s_target, g, partial);
    if (loss) hipLaunchKernelGGL(k_add_sum, dim3(1), dim3(256), 0, st, (const float*)partial, nb, loss);
    return hipGetLastError();
}

hipError_t launch_loss_finalize(const float* tile_sse, const SliceGeo* geo, int32_t m, const float* msum,
                                float* slice_sse, float* loss, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_sse, dim3(m), dim3(256), 0, st, tile_sse, geo, slice_sse);
    if (loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, (const float*)slice_sse, m, msum, loss);
    return hipGetLastError();
}

hipError_t launch_backward(const RenderArgs& a, const float* grad_pred, const float* grad_scale,
                           float4* inst_grad, int* work_counter, hipStream_t st) {
    if (a.n_tiles <= 0 || a.n_inst <= 0) return hipSuccess;
    // four waves per workgroup (one wave per tile measured slower: tiles with
    // many instances then serialise on a single wave)
    constexpr int NT = 256;
    if (a.persistent) {  // whole tiles, heaviest first, from a work queue
        hipError_t e = launch_fill_zero(work_counter, sizeof(int), st);
        if (e != hipSuccess) return e;
        const int grid = grid_for(a, NT);
        switch (a.tile) {
            case 8:
                hipLaunchKernelGGL((k_backward_tiles<8, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            case 16:
                hipLaunchKernelGGL((k_backward_tiles<16, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            case 32:
                hipLaunchKernelGGL((k_backward_tiles<32, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    // fixed chunks of 256 instances of the tile-ordered list
    const int64_t n_chunks = (a.n_inst + NT - 1) / NT;
    if (n_chunks > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    const int grid = (int)(((n_chunks + 7) >> 3) << 3);  // whole XCD remap
    switch (a.tile) {
        case 8:
            hipLaunchKernelGGL((k_backward<8, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        case 16:
            hipLaunchKernelGGL((k_backward<16, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        case 32:
            hipLaunchKernelGGL((k_backward<32, NT>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace svr
