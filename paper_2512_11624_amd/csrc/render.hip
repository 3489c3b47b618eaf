// Tile stages: per-tile instance ranges and the shape-class order of each
// tile's instances (the end of the binning), the forward accumulation with
// the masked-MSE epilogue, and the adjoint.  gfx950, wave64, FP32.
//
// Forward, pixel per lane (mode 0): a workgroup owns one T x T pixel tile of
// one slice.  Records of the tile are staged in LDS in batches; each wave owns
// a band of rows and skips records whose footprint rows miss its band.  The
// exponent of a record at tile-local pixel (X, Y) (relative to the tile
// centre) is the quadratic c0 + c1 X + c2 Y + c3 X^2 + c4 XY + c5 Y^2 whose
// coefficients are formed once per record at staging, so a pixel-record term
// costs 5 FMA, one exp2 and the window max(e - e_T, 0).  Every pixel sums its
// records in the sorted (deterministic) order.
//
// Forward, record per lane (mode 1, the default) and the adjoint: each lane
// owns one instance and walks its record's footprint box inside the tile.
// The binning orders every tile's instances by box shape, so the consecutive
// instances on a wave's lanes walk boxes of (nearly) one shape.  The forward
// adds fixed-point terms into an LDS pixel tile with integer atomics; the
// adjoint accumulates the seven moment sums it needs in registers (no
// cross-lane reduction) and writes them to the instance's emission slot (no
// atomics).  Both take fixed chunks of 256 instances of the tile-ordered list
// per workgroup, or (persistent) whole tiles from a work queue.
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kMaxBatch = 256;

__device__ inline int xcd_tile(int b, int n_tiles) {
    // consecutive tiles (which share records) go to the same XCD / L2
    const int per = (n_tiles + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// [start, end) of every tile's instances in the tile-sorted list; each
// thread looks at four consecutive keys.  Slots outside every tile (padding
// keys, sorted last) are copied to pad_out, the buffer the class order then
// fills, so that they keep their padding key there.
__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, int64_t n, int2* __restrict__ ranges,
                              uint32_t n_tiles, uint32_t* __restrict__ pad_out) {
    const int64_t s0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (s0 >= n) return;
    uint32_t key[4];
    uint32_t k[6];  // tile ids of keys s0 - 1 .. s0 + 4 (n_tiles outside the list)
    // the six loads in flight at once (indices clamped, results selected)
    uint32_t raw[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) raw[j] = keys[min(max(s0 - 1 + j, (int64_t)0), n - 1)];
    k[0] = s0 > 0 ? raw[0] >> kClassBits : n_tiles;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const uint32_t v = s0 + j < n ? raw[j + 1] : 0xffffffffu;
        if (j < 4) key[j] = v;
        k[j + 1] = s0 + j < n ? min(v >> kClassBits, n_tiles) : n_tiles;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t t = k[j + 1];
        if (s0 + j >= n) break;
        if (t >= n_tiles) {
            if (pad_out) pad_out[s0 + j] = key[j];
            continue;
        }
        if (k[j] != t) ranges[t].x = (int)(s0 + j);
        if (k[j + 2] != t) ranges[t].y = (int)(s0 + j + 1);
    }
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Block partial sums of x [n]: 16-byte loads for the aligned body.
__global__ __launch_bounds__(256) void k_partial_sum(const float* __restrict__ x, int64_t n,
                                                      float* __restrict__ partial) {
    __shared__ float s[4];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int head = (int)(((16 - ((uintptr_t)x & 15)) & 15) >> 2);  // scalars before the first 16-byte boundary
    const int64_t nh = head < n ? head : n;
    const int64_t n4 = (n - nh) >> 2;
    const float4* x4 = reinterpret_cast<const float4*>(x + nh);
    for (int64_t i = t0; i < n4; i += stride) {
        const float4 v = x4[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (t0 < nh) acc += x[t0];
    for (int64_t i = nh + 4 * n4 + t0; i < n; i += stride) acc += x[i];
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

// Forward walk of one instance's box inside its tile, rows outer and columns
// inner: adds round(amq max(e - e_T, 0)) to acc[y * T + x] (tile-local pixel)
// with an integer LDS atomic; pixels outside the cut add an integer zero
// (branch-free).  The term is amq e - amq e_T clamped (v_med3) to zero on the
// side opposite to amq's sign, rounded half up to an integer
// (v_cvt_rpi_i32_f32); the LDS address is the loop variable.  Returns the
// number of in-cut pixels when kCount.
__device__ inline int round_half_up(float v) {
    int q;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(q) : "v"(v));
    return q;
}

template <int T, bool kCount>
__device__ inline unsigned int forward_walk(const LaneBox& b, float amq, int* acc, float etau) {
    const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
    const int hh = w > 0 ? h : 0;
    const float dx0 = (float)b.x0 - b.pxl, b2a01 = 2.f * b.a01;
    const float c = -amq * etau;
    const float lo = amq >= 0.f ? 0.f : -__builtin_inff(), hi = amq >= 0.f ? __builtin_inff() : 0.f;
    float dy = (float)b.y0 - b.pyl;
    int* row = acc + b.y0 * T + b.x0;
    unsigned int cnt = 0;
    for (int r = 0; r < hh; ++r) {
        const float zy = fmaf(b.a11 * dy, dy, b.bz), bxl = b2a01 * dy;
        float dx = dx0;
        int* const end = row + w;
        for (int* p = row; p < end; ++p) {
            const float e = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(b.a00, dx, bxl), zy));
            atomicAdd(p, round_half_up(__builtin_amdgcn_fmed3f(fmaf(amq, e, c), lo, hi)));
            if (kCount) cnt += e > etau ? 1u : 0u;
            dx += 1.f;
        }
        dy += 1.f;
        row += T;
    }
    return cnt;
}

// The seven sums of one instance's adjoint, with t = g e inside the cut:
//   Sa = sum g max(e - e_T, 0), S0 = sum t, Sx = sum t dx, Sy = sum t dy,
//   Sxx = sum t dx^2, Sxy = sum t dx dy, Syy = sum t dy^2.
struct AdjointSums {
    float Sa, S0, Sx, Sy, Sxx, Sxy, Syy;
};

// Adjoint walk of one instance's box over the tile's upstream gradients g
// (T x T in LDS), rows outer and columns inner, with the per-row sums folded
// in with dy (three accumulations per pixel).
template <int T>
__device__ inline AdjointSums adjoint_walk(const LaneBox& b, const float* g, float etau, int stride = T) {
    const int w = max(b.x1 - b.x0 + 1, 0), h = max(b.y1 - b.y0 + 1, 0);
    const int hh = w > 0 ? h : 0;
    AdjointSums S = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float dx0 = (float)b.x0 - b.pxl, b2a01 = 2.f * b.a01;
    float dy = (float)b.y0 - b.pyl;
    int gr = b.y0 * stride + b.x0;
    for (int r = 0; r < hh; ++r) {
        const float zy = fmaf(b.a11 * dy, dy, b.bz), bxl = b2a01 * dy;
        float R0 = 0.f, R1 = 0.f, R2 = 0.f, dx = dx0;
        int gi = gr;
        for (int c = 0; c < w; ++c) {
            const float gv = g[gi];
            const float e = __builtin_amdgcn_exp2f(fmaf(dx, fmaf(b.a00, dx, bxl), zy));
            const float v = e - etau;
            const float gm = (v > 0.f) ? gv : 0.f;  // g inside the cut
            S.Sa = fmaf(gm, v, S.Sa);
            const float t = gm * e;
            const float tx = t * dx;
            R0 += t;
            R1 += tx;
            R2 = fmaf(tx, dx, R2);
            dx += 1.f;
            ++gi;
        }
        S.S0 += R0;
        S.Sx += R1;
        S.Sxx += R2;
        S.Sy = fmaf(dy, R0, S.Sy);
        S.Sxy = fmaf(dy, R1, S.Sxy);
        S.Syy = fmaf(dy * dy, R0, S.Syy);
        dy += 1.f;
        gr += stride;
    }
    return S;
}

// Gradient with respect to the stored record fields (dz/d field, times
// amp ln 2) from the seven sums, to the instance's emission slot.  The
// upstream scale multiplies every sum (it was not applied to g).
__device__ inline void store_adjoint(const AdjointSums& S, const LaneBox& b, float scale, float4* inst_grad,
                                     uint32_t e_slot) {
    const float k2 = b.am * SVR_LN2 * scale;
    float4 g0, g1;
    g0.x = S.Sa * scale;
    g0.y = k2 * S.S0;
    g0.z = -2.f * k2 * (b.a00 * S.Sx + b.a01 * S.Sy);
    g0.w = -2.f * k2 * (b.a01 * S.Sx + b.a11 * S.Sy);
    g1.x = k2 * S.Sxx;
    g1.y = 2.f * k2 * S.Sxy;
    g1.z = k2 * S.Syy;
    g1.w = 0.f;
    inst_grad[2 * (int64_t)e_slot] = g0;
    inst_grad[2 * (int64_t)e_slot + 1] = g1;
}

// Upstream gradients of one tile into LDS, T x T floats, zero outside the
// slice; 16-byte loads where a row's four pixels are inside the slice and
// aligned.
template <int T, int NT>
__device__ inline void stage_tile(const float* __restrict__ src, const TileOrg& o, float* dst) {
    constexpr int Q = T * T / 4;
    for (int q = threadIdx.x; q < Q; q += NT) {
        const int px = (q % (T / 4)) * 4, py = q / (T / 4);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (py < o.vh) {
            const int64_t gi = o.base + (int64_t)py * o.stride + px;
            if (px + 3 < o.vw && (gi & 3) == 0) {
                v = *reinterpret_cast<const float4*>(src + gi);
            } else {
                if (px < o.vw) v.x = src[gi];
                if (px + 1 < o.vw) v.y = src[gi + 1];
                if (px + 2 < o.vw) v.z = src[gi + 2];
                if (px + 3 < o.vw) v.w = src[gi + 3];
            }
        }
        *reinterpret_cast<float4*>(dst + py * T + px) = v;
    }
}

// Binning, last step: every tile's instances (sorted by tile, in emission
// order) are put in order of shape class, the low kClassBits of the key,
// stably, in segments of kSeg: one workgroup per tile ranks each instance
// within its class with ballot masks (lanes holding the same class) in input
// order, with per-wave class counters in LDS, places it in LDS and writes the
// segment out in order (coalesced).
// The record-per-lane tile kernels take consecutive instances on a wave's
// lanes, which then walk boxes of (nearly) one shape.
constexpr int kSeg = 4096;
static_assert(kClasses == 64, "one lane per class in the class scan");
__global__ __launch_bounds__(256) void k_class_order(const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ idx,
                                                     const int2* __restrict__ ranges, int32_t n_tiles,
                                                     uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                     uint32_t* __restrict__ idx_out) {
    constexpr int NT = 256, NW = 4, PER = kSeg / NT;  // wave w ranks [w PER 64, (w + 1) PER 64)
    __shared__ int s_cnt[NW][kClasses];
    __shared__ int s_start[kClasses];
    __shared__ uint32_t s_k[kSeg], s_v[kSeg], s_x[kSeg];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int tile = xcd_tile(blockIdx.x, n_tiles);
    if (tile >= n_tiles) return;
    const int2 rg = ranges[tile];
    const int n = rg.y - rg.x;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int s0 = 0; s0 < n; s0 += kSeg) {
        const int sn = min(kSeg, n - s0);
        const int64_t base = (int64_t)rg.x + s0;
        __syncthreads();  // the previous segment's counters are consumed
        s_cnt[wv][lane] = 0;
        __syncthreads();
        uint32_t kk[PER], vv[PER], xx[PER];
        int rk[PER];
        // a wave stops at its first iteration without entries (wave-uniform):
        // small tiles rank only the iterations they fill
        const int nit = min(PER, max(0, (sn - wv * PER * 64 + 63) >> 6));
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int j = wv * PER * 64 + it * 64 + lane;
            const bool valid = j < sn;
            kk[it] = valid ? keys[base + j] : 0u;
            vv[it] = valid ? vals[base + j] : 0u;
            xx[it] = valid ? idx[base + j] : 0u;
            rk[it] = -1;
        }
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            if (it >= nit) continue;  // wave-uniform
            const int j = wv * PER * 64 + it * 64 + lane;
            const bool valid = j < sn;
            const int c = (int)(kk[it] & (uint32_t)(kClasses - 1));
            uint64_t peers = __ballot(valid);
            for (int bit = 0; bit < kClassBits; ++bit) {
                const bool on = (c >> bit) & 1;
                const uint64_t bb = __ballot(on);
                peers &= on ? bb : ~bb;
            }
            if (!valid) peers = 0ull;
            const int leader = valid ? (__ffsll((long long)peers) - 1) : lane;
            int basec = 0;
            if (valid && lane == leader) {
                basec = s_cnt[wv][c];
                s_cnt[wv][c] = basec + __popcll(peers);
            }
            basec = __shfl(basec, leader, 64);
            rk[it] = valid ? basec + __popcll(peers & lt_mask) : -1;
        }
        __syncthreads();
        if (tid < 64) {  // class tid: prefix over waves, then the class starts
            int tot = 0;
            for (int q = 0; q < NW; ++q) {
                const int c = s_cnt[q][tid];
                s_cnt[q][tid] = tot;
                tot += c;
            }
            int incl = tot;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o) incl += u;
            }
            s_start[tid] = incl - tot;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            if (rk[it] >= 0) {
                const int c = (int)(kk[it] & (uint32_t)(kClasses - 1));
                const int d = s_start[c] + s_cnt[wv][c] + rk[it];
                s_k[d] = kk[it];
                s_v[d] = vv[it];
                s_x[d] = xx[it];
            }
        }
        __syncthreads();
        for (int j = tid; j < sn; j += NT) {
            keys_out[base + j] = s_k[j];
            vals_out[base + j] = s_v[j];
            idx_out[base + j] = s_x[j];
        }
    }
}

// Forward, record per lane, one tile per workgroup (persistent: tiles from
// the work queue, heaviest first), with exact integer accumulation.  Lane i
// takes the tile's instances i, i + 256, ... (in shape-class order from the
// binning) and walks each box (forward_walk).  The quantum comes from the
// tile alone: with 2^emax <= |a| < 2^(emax + 1) for the tile's largest
// amplitude and n instances, no pixel sum reaches 2^ex,
// ex = emax + 1 + ceil(log2 n), and 2^ex spans 2^30 quanta, so the int32 sums
// cannot overflow and a term's rounding error is below 2^-31 of n times the
// largest amplitude.  Integer sums do not depend on the order of the adds, so
// the result is deterministic.  A non-finite amplitude makes the tile's
// pixels NaN.
template <int T, bool kLoss, bool kCount>
__global__ __launch_bounds__(256) void k_forward_tiles(RenderArgs a, const float* __restrict__ target,
                                                      const float* __restrict__ mask,
                                                      const float* __restrict__ msum,
                                                      float* __restrict__ pred, float* __restrict__ grad,
                                                      float* __restrict__ tile_sse,
                                                      unsigned long long* __restrict__ incut,
                                                      int* __restrict__ work_counter) {
    constexpr int NT = 256, NW = 4;
    constexpr int kNoAmp = -100000;  // exponent sentinel: no nonzero amplitude
    __shared__ int s_acc[T * T];
    __shared__ int s_emax[NW];
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
        const int2 rg = a.ranges[tile];
        const int n = max(rg.y - rg.x, 0);
        const TileOrg o = tile_org(a.tile_org[tile]);
        __syncthreads();  // the previous tile is done with LDS
        for (int p = tid; p < T * T; p += NT) s_acc[p] = 0;
        // the tile's largest amplitude exponent (a max: order-independent)
        int emax = kNoAmp;
        bool bad = false;
        for (int j = tid; j < n; j += NT) {
            const float aa = fabsf(a.rec[a.inst_rec[rg.x + j]].r0.w);
            if (!(aa <= 3.4028235e38f)) bad = true;
            else if (aa > 0.f) emax = max(emax, ilogbf(aa));
        }
        for (int off = 32; off > 0; off >>= 1) emax = max(emax, __shfl_xor(emax, off, 64));
        const bool wbad = __ballot(bad) != 0ull;
        if (lane == 0) s_emax[wv] = wbad ? INT_MAX : emax;
        __syncthreads();
        int em = kNoAmp;
        bool tbad = false;
        for (int q = 0; q < NW; ++q) {
            const int v = s_emax[q];
            if (v == INT_MAX) tbad = true;
            else em = max(em, v);
        }
        const int lgn = n > 1 ? 32 - __clz((unsigned)(n - 1)) : 0;
        const int ex = em > kNoAmp ? em + 1 + lgn : 0;
        const int sh = min(max(30 - ex, -126), 126);
        const float to_q = ldexpf(1.f, sh), from_q = ldexpf(1.f, -sh);
        unsigned int cnt = 0;
        for (int j = tid; j < n; j += NT) {
            const Record R = a.rec[a.inst_rec[rg.x + j]];
            const LaneBox b = lane_box(R, o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
            cnt += forward_walk<T, kCount>(b, b.am * to_q, s_acc, etau);
        }
        __syncthreads();
        float sq = 0.f;
        for (int p = tid; p < T * T; p += NT) {
            const int px = p % T, py = p / T;
            if (px < o.vw && py < o.vh) {
                const int64_t pi = o.base + (int64_t)py * o.stride + px;
                const float y = tbad ? __builtin_nanf("") : (float)s_acc[p] * from_q;
                pred[pi] = y;
                if (kLoss) loss_term(a.loss_kind, mask[pi], y - target[pi], inv_msum, sq, grad ? grad + pi : nullptr);
            }
        }
        if (kLoss || kCount) {
            for (int off = 32; off > 0; off >>= 1) {
                sq += __shfl_xor(sq, off, 64);
                if (kCount) cnt += __shfl_xor(cnt, off, 64);
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
template <int T, int NT, bool kLoss, bool kPrefetch = false>
__device__ inline void finish_tile(const RenderArgs& a, int tile, const float* acc, const TileOrg& o,
                                   const float* __restrict__ target, const float* __restrict__ mask,
                                   float inv_msum, float* __restrict__ pred, float* __restrict__ grad,
                                   float* __restrict__ tile_sse, float* s_red) {
    const int tid = threadIdx.x;
    float sq = 0.f;
    if (kPrefetch) {
        // every target and mask load of the thread is issued before its first
        // store: a load issued after a store waits for the store as well
        constexpr int PPT = (T * T + NT - 1) / NT;
        float tv[PPT], mv[PPT];
        int64_t pix[PPT];
        bool in[PPT];
    #pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = tid + k * NT, px = p % T, py = p / T;
            in[k] = p < T * T && px < o.vw && py < o.vh;
            pix[k] = in[k] ? o.base + (int64_t)py * o.stride + px : o.base;  // the tile's first pixel is inside
            tv[k] = kLoss ? target[pix[k]] : 0.f;
            mv[k] = kLoss ? mask[pix[k]] : 0.f;
        }
    #pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (in[k]) {
                const float y = acc[tid + k * NT];
                pred[pix[k]] = y;
                if (kLoss) loss_term(a.loss_kind, mv[k], y - tv[k], inv_msum, sq, grad ? grad + pix[k] : nullptr);
            }
    } else {  // fewer registers where the caller holds many
        for (int p = tid; p < T * T; p += NT) {
            const int px = p % T, py = p / T;
            if (px < o.vw && py < o.vh) {
                const int64_t pi = o.base + (int64_t)py * o.stride + px;
                const float y = acc[p];
                pred[pi] = y;
                if (kLoss) loss_term(a.loss_kind, mask[pi], y - target[pi], inv_msum, sq, grad ? grad + pi : nullptr);
            }
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

// The chunked tile kernels give each workgroup 256 NI consecutive instances
// of the tile-ordered list; lane i takes instances i, i + 256, ...  The loads
// of a lane's NI instances are issued together, so their latency is paid once
// per NI instances (measured best: NI = 2 for the forward, 1 for the adjoint,
// whose walk holds more registers).
constexpr int kFwdPer = 2;
constexpr int kBwdPer = 1;

// Runs (distinct tiles) of a chunk: rslot[k] is the index of the run of the
// lane's k-th instance (chunk order: k, then wave, then lane), or -1 if it
// has none; returns the number of runs.  hm[k] are the wave's ballots of
// run heads.  Called by all threads; s_wsum [NI][4] scratch; ends with a
// barrier.
template <int NI>
__device__ inline int chunk_runs(const uint64_t* hm, const int* tile, const bool* head, int (*s_wsum)[4],
                                 int* rslot) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < NI; ++k)
        if (lane == 0) s_wsum[k][wv] = __popcll(hm[k]);
    __syncthreads();
    int run = 0, pre[NI];
    for (int k = 0; k < NI; ++k)
        for (int q = 0; q < 4; ++q) {
            if (q == wv) pre[k] = run;
            run += s_wsum[k][q];
        }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int k = 0; k < NI; ++k)
        rslot[k] = tile[k] >= 0 ? pre[k] + __popcll(hm[k] & lt) + (head[k] ? 1 : 0) - 1 : -1;
    return run;
}

// Forward, record per lane with exact integer accumulation, over fixed chunks
// of the tile-ordered instance list (the chunking of the adjoint): a chunk may
// span a few tiles.  The binning orders each tile's instances by footprint
// box shape, so the lanes of a wave walk boxes of (nearly) one shape.  Per
// pass (up to KT of the chunk's tiles) each lane walks its boxes
// (forward_walk) into its tile's int32 LDS sums.  The quantum is 2^(e - 30)
// with 2^e above the pass's sum of |a|, so no pixel's sum can overflow and the
// rounding error per term is below 2^-31 of that sum; integer sums do not
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
    constexpr int NT = 256, NW = 4, NI = kFwdPer, kChunk = NT * NI;
    constexpr int KT = (2048 * NI / (T * T)) > 0 ? 2048 * NI / (T * T) : 1;  // 8 NI KB of sums per pass
    __shared__ int s_iacc[KT * T * T];  // fixed-point sums, then (in place) their float values
    __shared__ int s_wsum[NI][NW];
    __shared__ float s_fsum[NW];
    __shared__ float s_red[NW];
    __shared__ unsigned int s_cnt[NW];
    __shared__ int4 s_org[KT];  // the pass's tiles (TileOrg packing)
    __shared__ int s_ptile[KT];
    __shared__ int s_fin[KT];  // -1: tile finished here, else the partial slot (0 first run, 1 last run)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n_chunks = (a.n_inst + kChunk - 1) / kChunk;
    const int64_t chunk = xcd_tile(blockIdx.x, (int)n_chunks);
    if (chunk >= n_chunks) return;  // idle workgroup of the XCD remap (uniform)
    const int64_t c0 = chunk * kChunk;
    const float etau = a.etau;
    const float tau2k = SVR_KZ * a.tau2;
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    float* s_facc = reinterpret_cast<float*>(s_iacc);

    // the lane's instances: tile, run head, record and box.  The loads come
    // in two dependent rounds, each issued at once and without branches
    // (indices clamped, results selected): keys (the instance's and its
    // predecessor's) and record ids; then records, tile origins and ranges.
    int tile[NI], fin[NI], rslot[NI];
    bool head[NI];
    int4 org[NI];
    uint64_t hm[NI];
    LaneBox b[NI];
    uint32_t key[NI], kprev[NI], rid[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t inst = c0 + k * NT + tid;
        const int64_t ic = min(inst, a.n_inst - 1);
        key[k] = a.inst_key[ic];
        kprev[k] = a.inst_key[ic > 0 ? ic - 1 : 0];
        rid[k] = a.inst_rec[ic];
    }
    __builtin_amdgcn_sched_barrier(0);
    Record R[NI];
    int2 rg[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t inst = c0 + k * NT + tid;
        const uint32_t t = inst < a.n_inst ? key[k] >> kClassBits : ~0u;
        const bool live = t < (uint32_t)a.n_tiles;
        tile[k] = live ? (int)t : -1;
        head[k] = live && (inst == c0 || (kprev[k] >> kClassBits) != t);
        R[k] = a.rec[live ? rid[k] : 0u];
        org[k] = a.tile_org[live ? t : 0u];
        rg[k] = a.ranges[live ? t : 0u];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t inst = c0 + k * NT + tid;
        b[k] = LaneBox{};
        fin[k] = -1;
        if (tile[k] >= 0) {
            const TileOrg o = tile_org(org[k]);
            b[k] = lane_box(R[k], o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
            if (head[k]) {
                const bool inside = rg[k].x >= c0 && rg[k].y <= c0 + kChunk;
                fin[k] = inside ? -1 : (inst == c0 ? 0 : 1);
            }
        }
        hm[k] = __ballot(head[k]);
    }
    const int nd = chunk_runs<NI>(hm, tile, head, s_wsum, rslot);
    unsigned int cnt = 0;
    for (int p0 = 0; p0 < nd; p0 += KT) {
        const int np = min(KT, nd - p0);
        if (p0 > 0) __syncthreads();  // the previous pass is done with LDS
        float pa = 0.f;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const bool act = rslot[k] >= p0 && rslot[k] < p0 + np;
            if (act && head[k]) {
                s_org[rslot[k] - p0] = org[k];
                s_ptile[rslot[k] - p0] = tile[k];
                s_fin[rslot[k] - p0] = fin[k];
            }
            if (act && b[k].x1 >= b[k].x0 && b[k].y1 >= b[k].y0) pa += fabsf(b[k].am);
        }
        for (int q = tid; q < np * T * T; q += NT) s_iacc[q] = 0;
        // the pass's sum of |a| (its instances only)
        for (int off = 32; off > 0; off >>= 1) pa += __shfl_xor(pa, off, 64);
        if (lane == 0) s_fsum[wv] = pa;
        __syncthreads();
        const float suma = (s_fsum[0] + s_fsum[1]) + (s_fsum[2] + s_fsum[3]);
        // quantum: the pass's sum of |a| spans 2^30 quanta.  A non-finite
        // amplitude has no quantum: the pass's pixels become NaN below.
        const bool bad = !(suma <= 3.4028235e38f);
        const int ex = (suma > 0.f && !bad) ? ilogbf(suma) + 1 : 0;
        const float to_q = ldexpf(1.f, 30 - ex);
#pragma unroll
        for (int k = 0; k < NI; ++k)
            if (rslot[k] >= p0 && rslot[k] < p0 + np)
                cnt += forward_walk<T, kCount>(b[k], b[k].am * to_q, s_iacc + (rslot[k] - p0) * T * T, etau);
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
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
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
    constexpr int NT = 256, kChunk = NT * kFwdPer;
    __shared__ float s_acc[T * T];
    __shared__ float s_red[NT / 64];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    const int2 rg = a.ranges[tile];
    const int64_t c0 = rg.y > rg.x ? rg.x / kChunk : 0, c1 = rg.y > rg.x ? (rg.y - 1) / kChunk : -1;
    if (rg.y > rg.x && c0 == c1) return;  // finished by its chunk
    const float inv_msum = (kLoss && msum[0] > 0.f) ? 1.f / msum[0] : 0.f;
    // every thread's pixels, summed over the chunks in chunk order; the loads
    // of eight chunks are issued together
    constexpr int PPT = (T * T + NT - 1) / NT;
    constexpr int U = 8;
    float acc[PPT];
    for (int k = 0; k < PPT; ++k) acc[k] = 0.f;
    for (int64_t cb = c0; cb <= c1; cb += U) {
        float v[U][PPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = cb + u;
            const int ps = (c == c0 && rg.x != c0 * kChunk) ? 1 : 0;
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
    finish_tile<T, NT, kLoss, true>(a, tile, s_acc, tile_org(a.tile_org[tile]), target, mask, inv_msum, pred, grad,
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
// The binning orders a tile's instances by box shape, so the four groups of
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

// Adjoint, record per lane, one tile per workgroup (persistent: tiles from
// the work queue, heaviest first).  The tile's upstream gradients are staged
// in LDS once; lane i takes the tile's instances i, i + 256, ... (in
// shape-class order from the binning), walks each box (adjoint_walk) and
// writes the gradient to the instance's emission slot: no cross-lane
// reduction and no atomics, so the result is deterministic.
template <int T>
__global__ __launch_bounds__(256) void k_backward_tiles(RenderArgs a, const float* __restrict__ grad_pred,
                                                       const float* __restrict__ grad_scale,
                                                       float4* __restrict__ inst_grad,
                                                       int* __restrict__ work_counter) {
    constexpr int NT = 256;
    __shared__ __align__(16) float s_g[T * T];
    __shared__ int s_next;
    const int tid = threadIdx.x;
    const float tau2k = SVR_KZ * a.tau2;
    const float scale = grad_scale ? grad_scale[0] : 1.f;
    int iter = 0;
    while (true) {
        const int tile = next_tile<NT>(a, work_counter, iter, &s_next);
        if (tile < 0) break;
        const int2 rg = a.ranges[tile];
        const int n = rg.y - rg.x;
        if (n <= 0) continue;
        const TileOrg o = tile_org(a.tile_org[tile]);
        __syncthreads();  // the previous tile is done with s_g
        stage_tile<T, NT>(grad_pred, o, s_g);
        __syncthreads();
        for (int j = tid; j < n; j += NT) {
            const int64_t i = rg.x + j;
            const Record R = a.rec[a.inst_rec[i]];
            const uint32_t e_slot = a.inst_idx[i];
            const LaneBox b = lane_box(R, o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
            store_adjoint(adjoint_walk<T>(b, s_g, a.etau), b, scale, inst_grad, e_slot);
        }
    }
}

// Adjoint, record per lane, over fixed chunks of the tile-ordered instance
// list (256 kBwdPer instances, kBwdPer per lane, which may span a few tiles).
// The binning orders each tile's instances by footprint box shape, so the 64
// consecutive instances a wave takes walk boxes of (nearly) one shape.  When
// the chunk's instances lie in at most KT consecutive tiles, or in just its
// first and last tile (the usual cases), their upstream gradients are staged
// in LDS at once, while the lanes' record loads are in flight; otherwise in
// passes of up to KT of the chunk's tiles.  Each lane walks its records'
// boxes (adjoint_walk) and writes each instance's gradient to its emission
// slot: no cross-lane reduction and no atomics, so the result is
// deterministic and independent of the chunking.
template <int T>
__global__ __launch_bounds__(256, 8) void k_backward(RenderArgs a, const float* __restrict__ grad_pred,
                                                    const float* __restrict__ grad_scale,
                                                    float4* __restrict__ inst_grad) {
    constexpr int NT = 256, NI = kBwdPer, kChunk = NT * NI;
    constexpr int KT = 2048 / (T * T) > 0 ? 2048 / (T * T) : 1;  // tiles staged (8 KB)
    constexpr int Q = T * T / 4;                                   // float4 per tile
    constexpr int NS = (KT * Q + NT - 1) / NT;                     // staged float4 per thread
    __shared__ __align__(16) float s_g[KT * T * T];
    __shared__ int s_wsum[NI][4];
    __shared__ int4 s_org[KT];  // a pass's tiles (TileOrg packing)
    __shared__ int s_other[4];  // per wave: a lane's tile is neither tf nor tl
    const int tid = threadIdx.x;
    const int64_t n_chunks = (a.n_inst + kChunk - 1) / kChunk;
    const int64_t chunk = xcd_tile(blockIdx.x, (int)n_chunks);
    if (chunk >= n_chunks) return;  // idle workgroup of the XCD remap (uniform)
    const int64_t c0 = chunk * kChunk;
    const float tau2k = SVR_KZ * a.tau2;
    const float scale = grad_scale ? grad_scale[0] : 1.f;

    // Loads in three dependent rounds, each issued at once and without
    // branches (indices clamped, results selected): (1) the chunk's first and
    // last keys and the lane's keys, record ids and emission slots; (2) the
    // lane's records and tile origins, and the origins of the tiles to stage;
    // (3) the staged upstream gradients.
    const uint32_t kf = a.inst_key[c0], kl = a.inst_key[min(c0 + kChunk, a.n_inst) - 1];
    uint32_t key[NI], rid[NI], e_slot[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t ic = min(c0 + k * NT + tid, a.n_inst - 1);
        key[k] = a.inst_key[ic];
        rid[k] = a.inst_rec[ic];
        e_slot[k] = a.inst_idx[ic];
    }
    __builtin_amdgcn_sched_barrier(0);
    // Staged slots: the chunk's tiles tf..tl when they are at most KT
    // consecutive ids ("range"), else tf and tl in slots 0 and 1 ("pair"),
    // which serves when every instance's tile is one of the two (checked
    // after the staging barrier); otherwise the runs of tiles go in passes.
    const uint32_t tf = kf >> kClassBits, tl = kl >> kClassBits;
    const bool valid_ends = tf < (uint32_t)a.n_tiles && tl < (uint32_t)a.n_tiles;
    const bool range = valid_ends && tl - tf < (uint32_t)KT;
    const bool pair = valid_ends && !range;
    const int nslot = range ? (int)(tl - tf) + 1 : (pair ? 2 : 0);
    // staged float4 q: slot q / Q, row and column of q % Q (at T = 32 a
    // thread's s-th float4 lies in slot s, whose origin is then uniform).
    // Without slots tf and tl may be padding keys (above every tile id):
    // stage loads then read tile 0, a real tile, and are unused.
    int4 ov[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int sl = Q >= NT ? s : (tid + s * NT) / Q;
        const uint32_t ts = range ? min(tf + (uint32_t)sl, tl) : (sl == 0 ? tf : tl);
        ov[s] = a.tile_org[nslot > 0 ? ts : 0u];
    }
    uint32_t t[NI];
    Record R[NI];
    int4 org[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        t[k] = c0 + k * NT + tid < a.n_inst ? key[k] >> kClassBits : ~0u;
        const bool live = t[k] < (uint32_t)a.n_tiles;
        R[k] = a.rec[live ? rid[k] : 0u];
        org[k] = a.tile_org[live ? t[k] : 0u];
    }
    __builtin_amdgcn_sched_barrier(0);
    // a tile whole inside its slice and 16-byte aligned (the usual case)
    // takes one 16-byte load per float4, others four clamped loads
    float4 sv[NS];
    const int nq = nslot * Q;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = tid + s * NT;
        const int64_t base = (int64_t)(((uint64_t)(uint32_t)ov[s].y << 32) | (uint64_t)(uint32_t)ov[s].x);
        const int stride = ov[s].w & 0xffff, vw = (ov[s].w >> 16) & 0xff, vh = (int)((uint32_t)ov[s].w >> 24);
        const int qq = q % Q, px = (qq % (T / 4)) * 4, py = qq / (T / 4);
        const float* row = grad_pred + base + (int64_t)min(py, vh - 1) * stride;
        const bool use = q < nq;
        if (vw == T && vh == T && ((base | stride) & 3) == 0) {
            const float4 v = *reinterpret_cast<const float4*>(row + px);
            sv[s] = use ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            const float x = row[min(px, vw - 1)], y = row[min(px + 1, vw - 1)];
            const float z = row[min(px + 2, vw - 1)], w = row[min(px + 3, vw - 1)];
            const bool in = use && py < vh;
            sv[s] = make_float4(in && px < vw ? x : 0.f, in && px + 1 < vw ? y : 0.f, in && px + 2 < vw ? z : 0.f,
                                in && px + 3 < vw ? w : 0.f);
        }
    }
    if (nslot > 0) {
        // float4 q of the staged slots sits at s_g[4 q] (slot q / Q, row and
        // column of q % Q)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = tid + s * NT;
            if (q < nq) *reinterpret_cast<float4*>(s_g + 4 * q) = sv[s];
        }
        bool other = false;
#pragma unroll
        for (int k = 0; k < NI; ++k) other |= t[k] < (uint32_t)a.n_tiles && t[k] != tf && t[k] != tl;
        const bool wave_other = __any(other);
        if ((tid & 63) == 0) s_other[tid >> 6] = wave_other ? 1 : 0;
        __syncthreads();
        if (range || !(s_other[0] | s_other[1] | s_other[2] | s_other[3])) {  // uniform
#pragma unroll
            for (int k = 0; k < NI; ++k)
                if (t[k] < (uint32_t)a.n_tiles) {
                    const TileOrg o = tile_org(org[k]);
                    const LaneBox b = lane_box(R[k], o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
                    const int slot = range ? (int)(t[k] - tf) : (t[k] == tf ? 0 : 1);
                    store_adjoint(adjoint_walk<T>(b, s_g + slot * T * T, a.etau), b, scale, inst_grad, e_slot[k]);
                }
            return;
        }
    }
    // the chunk holds more than two tiles that are not KT consecutive ids
    // (rare): its runs of tiles are staged in passes of KT (the barrier in
    // chunk_runs orders them after the staging above); each lane's record
    // and tile origin are reloaded (cached) when its pass comes rather than
    // held in registers
    int tile[NI], rslot[NI];
    bool head[NI];
    uint64_t hm[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t inst = c0 + k * NT + tid;
        const bool live = t[k] < (uint32_t)a.n_tiles;
        tile[k] = live ? (int)t[k] : -1;
        head[k] = live && (inst == c0 || (a.inst_key[inst - 1] >> kClassBits) != t[k]);
        hm[k] = __ballot(head[k]);
    }
    const int nd = chunk_runs<NI>(hm, tile, head, s_wsum, rslot);
    for (int p0 = 0; p0 < nd; p0 += KT) {
        const int np = min(KT, nd - p0);
        if (p0 > 0) __syncthreads();  // the previous pass is done with LDS
#pragma unroll
        for (int k = 0; k < NI; ++k)
            if (head[k] && rslot[k] >= p0 && rslot[k] < p0 + np) s_org[rslot[k] - p0] = a.tile_org[t[k]];
        __syncthreads();
        for (int sl = 0; sl < np; ++sl) stage_tile<T, NT>(grad_pred, tile_org(s_org[sl]), s_g + sl * T * T);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; ++k)
            if (rslot[k] >= p0 && rslot[k] < p0 + np) {
                const TileOrg o = tile_org(a.tile_org[t[k]]);
                const LaneBox b = lane_box(a.rec[rid[k]], o.x0, o.y0, o.vw - 1, o.vh - 1, tau2k);
                store_adjoint(adjoint_walk<T>(b, s_g + (rslot[k] - p0) * T * T, a.etau), b, scale, inst_grad,
                              e_slot[k]);
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
                              uint32_t* pad_out, hipStream_t st) {
    hipError_t e = launch_fill_zero(ranges, sizeof(int2) * (size_t)n_tiles, st);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((n + 1023) / 1024)), dim3(256), 0, st, keys, n, ranges,
                       (uint32_t)n_tiles, pad_out);
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
hipError_t fwd_tiles_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                              float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                              int* work_counter, int grid, hipStream_t st) {
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    if (loss && count)
        hipLaunchKernelGGL((k_forward_tiles<T, true, true>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else if (loss)
        hipLaunchKernelGGL((k_forward_tiles<T, true, false>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else if (count)
        hipLaunchKernelGGL((k_forward_tiles<T, false, true>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    else
        hipLaunchKernelGGL((k_forward_tiles<T, false, false>), dim3(grid), dim3(256), 0, st, a, target, mask, msum,
                           pred, grad, tile_sse, incut, work_counter);
    return hipGetLastError();
}

template <int T>
hipError_t fwd_chunk_dispatch(const RenderArgs& a, const float* target, const float* mask, const float* msum,
                              float* pred, float* grad, float* tile_sse, unsigned long long* incut,
                              float* partial, hipStream_t st) {
    const bool loss = target != nullptr;
    const bool count = incut != nullptr;
    constexpr int NT = 256, kChunk = NT * kFwdPer;
    const int64_t n_chunks = (a.n_inst + kChunk - 1) / kChunk;
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
    const int64_t n_chunks = (a.n_inst + 256 * kFwdPer - 1) / (256 * kFwdPer);
    return (size_t)n_chunks * 2 * (size_t)a.tile * (size_t)a.tile;
}

hipError_t launch_class_order(const uint32_t* keys, const uint32_t* vals, const uint32_t* idx, const int2* ranges,
                              int32_t n_tiles, uint32_t* keys_out, uint32_t* vals_out, uint32_t* idx_out,
                              hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    const int grid = ((n_tiles + 7) >> 3) << 3;  // whole XCD remap
    hipLaunchKernelGGL(k_class_order, dim3(grid), dim3(256), 0, st, keys, vals, idx, ranges, n_tiles, keys_out,
                       vals_out, idx_out);
    return hipGetLastError();
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
    if (a.forward_mode == 1 && !a.persistent) {
        switch (a.tile) {
            case 8: return fwd_chunk_dispatch<8>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            case 16: return fwd_chunk_dispatch<16>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            case 32: return fwd_chunk_dispatch<32>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, partial, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.forward_mode == 1) {
        const int grid = grid_for(a, 256);
        switch (a.tile) {
            case 8: return fwd_tiles_dispatch<8>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 16: return fwd_tiles_dispatch<16>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
            case 32: return fwd_tiles_dispatch<32>(a, target, mask, msum, pred, grad_pred, tile_sse, incut, work_counter, grid, st);
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
    constexpr int NT = 256;
    if (a.persistent) {  // whole tiles, heaviest first, from a work queue
        hipError_t e = launch_fill_zero(work_counter, sizeof(int), st);
        if (e != hipSuccess) return e;
        const int grid = grid_for(a, NT);
        switch (a.tile) {
            case 8:
                hipLaunchKernelGGL((k_backward_tiles<8>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            case 16:
                hipLaunchKernelGGL((k_backward_tiles<16>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            case 32:
                hipLaunchKernelGGL((k_backward_tiles<32>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad, work_counter);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    // fixed chunks of 256 kBwdPer instances of the tile-ordered list
    const int64_t n_chunks = (a.n_inst + NT * kBwdPer - 1) / (NT * kBwdPer);
    if (n_chunks > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    const int grid = (int)(((n_chunks + 7) >> 3) << 3);  // whole XCD remap
    switch (a.tile) {
        case 8:
            hipLaunchKernelGGL((k_backward<8>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        case 16:
            hipLaunchKernelGGL((k_backward<16>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        case 32:
            hipLaunchKernelGGL((k_backward<32>), dim3(grid), dim3(NT), 0, st, a, grad_pred, grad_scale, inst_grad);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace svr
