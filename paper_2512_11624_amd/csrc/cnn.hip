// Pose-proposal CNN on BF16 MFMA (gfx950): 6 x [3x3 conv, stride 2, pad 1,
// ReLU] with channels 32, 32, 64, 64, 128, 128 on a 1x128x128 crop, then
// FC 524 -> 256 (ReLU) -> 6 on the flattened 128x2x2 features concatenated
// with the slice's nominal placement (stack rotation R0, 9 floats, and the
// nominal centre t0 / 16 mm, 3 floats).  Every convolution and linear layer
// -- forward, input gradient and weight gradient -- is an implicit GEMM on
// v_mfma_f32_16x16x32_bf16 (the input gradient of the large layers is four:
// one per parity class of the input pixel, which drops the stride's zero
// taps): operands are rounded to BF16 (round to nearest even) when staged
// into LDS, products accumulate in FP32, master weights and activations stay
// FP32.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <vector>

#include "svr.h"
#include "svr_internal.h"

namespace svr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 32;

// C[M][N] = sum_k A[M][K] B[K][N].  Each thread stages 8 consecutive k of
// one row of A and one column of B per K step: a loader's prep(r) decodes
// that row (column) once, and load8(state, k0, v) fetches k0 .. k0 + 7 with
// the index walked incrementally (0 outside the operand).  The K loop is
// double-buffered: the next step's operands are fetched into registers
// while the current step's MFMAs run on the other LDS buffer, one barrier
// per step.  blockIdx.z selects the K range [z kz, (z+1) kz) (kz a multiple
// of BK): with several ranges (split K) the epilogue stores partial sums and
// a second kernel adds them in a fixed order.
template <class LA, class LB, class EP>
__global__ __launch_bounds__(256) void k_gemm(LA la, LB lb, EP ep, int M, int N, int K, int kz) {
    __shared__ __attribute__((aligned(16))) unsigned short sA[2][BM][BK];
    __shared__ __attribute__((aligned(16))) unsigned short sB[2][BN][BK];  // transposed: [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    floatx4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;  // staging: row / column lr, k offset lk
    const int kb = blockIdx.z * kz, ke = min(K, kb + kz);
    const auto sa = la.prep(m0 + lr);
    const auto sb = lb.prep(n0 + lr);
    float va[8], vb[8];
    if (kb < ke) {
        la.load8(sa, kb + lk, va);
        lb.load8(sb, kb + lk, vb);
    }
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK, buf ^= 1) {
        bf16x8 ua, ub;  // round to nearest even (v_cvt_pk_bf16_f32)
        for (int e = 0; e < 8; ++e) {
            ua[e] = (__bf16)va[e];
            ub[e] = (__bf16)vb[e];
        }
        *reinterpret_cast<bf16x8*>(&sA[buf][lr][lk]) = ua;
        *reinterpret_cast<bf16x8*>(&sB[buf][lr][lk]) = ub;
        __syncthreads();
        if (k0 + BK < ke) {  // next step's operands, in flight during this step's MFMAs
            la.load8(sa, k0 + BK + lk, va);
            lb.load8(sb, k0 + BK + lk, vb);
        }
        const int ko = 8 * (lane >> 4);
        for (int i = 0; i < 2; ++i) {
            const us8 a = *reinterpret_cast<const us8*>(&sA[buf][wm * 32 + i * 16 + (lane & 15)][ko]);
            for (int j = 0; j < 2; ++j) {
                const us8 b = *reinterpret_cast<const us8*>(&sB[buf][wn * 32 + j * 16 + (lane & 15)][ko]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                                    __builtin_bit_cast(bf16x8, b), acc[i][j], 0, 0, 0);
            }
        }
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) ep(row, col, acc[i][j][r]);
            }
}

// ---- convolution 3x3, stride 2, pad 1, NCHW, OH = (H+1)/2 --------------------
struct ConvShape {
    int B, Ci, H, W, Co, OH, OW;
};

// (c, kh, kw) of k = (c * 3 + kh) * 3 + kw, and the step to k + 1
struct Tap {
    int c, kh, kw;
};
__device__ inline Tap tap_of(int k) {
    const int t = k / 3;
    return Tap{t / 3, t - 3 * (t / 3), k - 3 * t};
}
__device__ inline void tap_next(Tap& t) {
    if (++t.kw == 3) {
        t.kw = 0;
        if (++t.kh == 3) {
            t.kh = 0;
            ++t.c;
        }
    }
}
// (n, y, x) of a raster index m = (n * Y + y) * X + x, and the step to m + 1
struct Pix {
    int n, y, x;
};
__device__ inline Pix pix_of(int m, int Y, int X) {
    const int t = m / X;
    return Pix{t / Y, t - Y * (t / Y), m - X * t};
}
__device__ inline void pix_next(Pix& p, int Y, int X) {
    if (++p.x == X) {
        p.x = 0;
        if (++p.y == Y) {
            p.y = 0;
            ++p.n;
        }
    }
}

// upstream gradient through the ReLU (mask = output > 0; out NULL = identity)
__device__ inline float dmask(const float* dy, const float* out, int64_t idx) {
    const float g = dy[idx];
    return (out && !(out[idx] > 0.f)) ? 0.f : g;
}

// forward: A = im2col(in) [B*OH*OW][Ci*9], B = W^T
struct LConvIn {
    const float* x;
    ConvShape s;
    struct St {
        const float* img;  // the row's image, channel 0
        int ih0, iw0;      // top-left input pixel of the 3x3 window
        bool ok;
    };
    __device__ St prep(int m) const {
        St r{x, 0, 0, m < s.B * s.OH * s.OW};
        if (r.ok) {
            const Pix p = pix_of(m, s.OH, s.OW);
            r.img = x + (int64_t)p.n * s.Ci * s.H * s.W;
            r.ih0 = 2 * p.y - 1;
            r.iw0 = 2 * p.x - 1;
        }
        return r;
    }
    __device__ void load8(const St& r, int k0, float* v) const {
        Tap t = tap_of(k0);
        const int kc = s.Ci * 9;
        for (int e = 0; e < 8; ++e) {
            const int ih = r.ih0 + t.kh, iw = r.iw0 + t.kw;
            const bool in = r.ok && k0 + e < kc && ih >= 0 && ih < s.H && iw >= 0 && iw < s.W;
            v[e] = in ? r.img[((int64_t)t.c * s.H + ih) * s.W + iw] : 0.f;
            tap_next(t);
        }
    }
};
struct LConvW {  // B[k][co] = W[co][k]
    const float* w;
    int Co, Kc;
    struct St {
        const float* p;
        bool ok;
    };
    __device__ St prep(int co) const { return St{w + (int64_t)min(co, Co - 1) * Kc, co < Co}; }
    __device__ void load8(const St& r, int k0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = (r.ok && k0 + e < Kc) ? r.p[k0 + e] : 0.f;
    }
};
struct EConvOut {
    float* y;
    const float* bias;
    ConvShape s;
    int relu;
    __device__ void operator()(int m, int co, float v) const {
        const int ow = m % s.OW, t = m / s.OW, oh = t % s.OH, n = t / s.OH;
        v += bias ? bias[co] : 0.f;
        if (relu) v = fmaxf(v, 0.f);
        y[(((int64_t)n * s.Co + co) * s.OH + oh) * s.OW + ow] = v;
    }
};

// input gradient: A[m=(n,ih,iw)][k=(co,kh,kw)] = dOut at oh = (ih+1-kh)/2 when integral
struct LConvDOut {
    const float* dy;
    const float* out;
    ConvShape s;
    struct St {
        int64_t base;  // offset of the row's sample, channel 0
        int ph0, pw0;  // ih + 1, iw + 1
        bool ok;
    };
    __device__ St prep(int m) const {
        St r{0, 0, 0, m < s.B * s.H * s.W};
        if (r.ok) {
            const Pix p = pix_of(m, s.H, s.W);
            r.base = (int64_t)p.n * s.Co * s.OH * s.OW;
            r.ph0 = p.y + 1;
            r.pw0 = p.x + 1;
        }
        return r;
    }
    __device__ void load8(const St& r, int k0, float* v) const {
        Tap t = tap_of(k0);
        const int kc = s.Co * 9;
        for (int e = 0; e < 8; ++e) {
            const int ph = r.ph0 - t.kh, pw = r.pw0 - t.kw;
            const int oh = ph >> 1, ow = pw >> 1;
            const bool in = r.ok && k0 + e < kc && ph >= 0 && pw >= 0 && !(ph & 1) && !(pw & 1) && oh < s.OH &&
                            ow < s.OW;
            v[e] = in ? dmask(dy, out, r.base + ((int64_t)t.c * s.OH + oh) * s.OW + ow) : 0.f;
            tap_next(t);
        }
    }
};
struct LConvWT {  // B[k=(co,kh,kw)][ci] = W[co][ci][kh][kw]
    const float* w;
    ConvShape s;
    struct St {
        const float* p;  // W[0][ci]
        bool ok;
    };
    __device__ St prep(int ci) const { return St{w + (int64_t)min(ci, s.Ci - 1) * 9, ci < s.Ci}; }
    __device__ void load8(const St& r, int k0, float* v) const {
        int co = k0 / 9, kk = k0 - 9 * co;
        const int kc = s.Co * 9;
        for (int e = 0; e < 8; ++e) {
            v[e] = (r.ok && k0 + e < kc) ? r.p[(int64_t)co * s.Ci * 9 + kk] : 0.f;
            if (++kk == 9) {
                kk = 0;
                ++co;
            }
        }
    }
};
struct EConvDIn {
    float* dx;
    ConvShape s;
    __device__ void operator()(int m, int ci, float v) const {
        const int iw = m % s.W, t = m / s.W, ih = t % s.H, n = t / s.H;
        dx[(((int64_t)n * s.Ci + ci) * s.H + ih) * s.W + iw] = v;
    }
};

// Input gradient split by the parity (py, px) of the input pixel: with
// stride 2, pixel ih = 2 y + py receives only from kernel rows kh with
// ih + 1 - kh even -- kh = 1 (oh = y) when py = 0, kh = 0 (oh = y + 1) and
// kh = 2 (oh = y) when py = 1 -- and likewise for columns.  The four classes
// are dense GEMMs over 1, 2, 2 and 4 taps per output channel (9 in all,
// against 9 per pixel for the plain implicit GEMM, whose other taps are
// zero).  Rows m = (n, y, x) of the class, k = (co, th, tw).
struct DgradClass {
    int py, px, nth, ntw, Hc, Wc;
};
__device__ inline int class_kh(int p, int t) { return p ? (t ? 2 : 0) : 1; }
struct LConvDOutP {
    const float* dy;
    const float* out;
    ConvShape s;
    DgradClass c;
    struct St {
        int64_t base;
        int y, x;
        bool ok;
    };
    __device__ St prep(int m) const {
        St r{0, 0, 0, m < s.B * c.Hc * c.Wc};
        if (r.ok) {
            const Pix p = pix_of(m, c.Hc, c.Wc);
            r.base = (int64_t)p.n * s.Co * s.OH * s.OW;
            r.y = p.y;
            r.x = p.x;
        }
        return r;
    }
    __device__ void load8(const St& r, int k0, float* v) const {
        const int nt = c.nth * c.ntw, kc = s.Co * nt;
        int co = k0 / nt, t = k0 - co * nt;
        int th = t / c.ntw, tw = t - th * c.ntw;
        for (int e = 0; e < 8; ++e) {
            const int oh = r.y + ((c.py && th == 0) ? 1 : 0), ow = r.x + ((c.px && tw == 0) ? 1 : 0);
            const bool in = r.ok && k0 + e < kc && oh < s.OH && ow < s.OW;
            v[e] = in ? dmask(dy, out, r.base + ((int64_t)co * s.OH + oh) * s.OW + ow) : 0.f;
            if (++tw == c.ntw) {
                tw = 0;
                if (++th == c.nth) {
                    th = 0;
                    ++co;
                }
            }
        }
    }
};
struct LConvWTP {  // B[k=(co,th,tw)][ci] = W[co][ci][kh(th)][kw(tw)]
    const float* w;
    ConvShape s;
    DgradClass c;
    struct St {
        const float* p;  // W[0][ci]
        bool ok;
    };
    __device__ St prep(int ci) const { return St{w + (int64_t)min(ci, s.Ci - 1) * 9, ci < s.Ci}; }
    __device__ void load8(const St& r, int k0, float* v) const {
        const int nt = c.nth * c.ntw, kc = s.Co * nt;
        int co = k0 / nt, t = k0 - co * nt;
        int th = t / c.ntw, tw = t - th * c.ntw;
        for (int e = 0; e < 8; ++e) {
            v[e] = (r.ok && k0 + e < kc) ? r.p[(int64_t)co * s.Ci * 9 + class_kh(c.py, th) * 3 + class_kh(c.px, tw)]
                                         : 0.f;
            if (++tw == c.ntw) {
                tw = 0;
                if (++th == c.nth) {
                    th = 0;
                    ++co;
                }
            }
        }
    }
};
struct EConvDInP {
    float* dx;
    ConvShape s;
    DgradClass c;
    __device__ void operator()(int m, int ci, float v) const {
        const Pix p = pix_of(m, c.Hc, c.Wc);
        const int ih = 2 * p.y + c.py, iw = 2 * p.x + c.px;
        dx[(((int64_t)p.n * s.Ci + ci) * s.H + ih) * s.W + iw] = v;
    }
};

// weight gradient: M = Co, N = Ci*9 (+1 bias column), K = B*OH*OW
struct LConvDOutT {  // A[co][m] = masked dOut, m = (n, oh, ow)
    const float* dy;
    const float* out;
    ConvShape s;
    struct St {
        int co;
        bool ok;
    };
    __device__ St prep(int co) const { return St{co, co < s.Co}; }
    __device__ void load8(const St& r, int m0, float* v) const {
        Pix p = pix_of(m0, s.OH, s.OW);
        const int mk = s.B * s.OH * s.OW;
        for (int e = 0; e < 8; ++e) {
            const bool in = r.ok && m0 + e < mk;
            v[e] = in ? dmask(dy, out, (((int64_t)p.n * s.Co + r.co) * s.OH + p.y) * s.OW + p.x) : 0.f;
            pix_next(p, s.OH, s.OW);
        }
    }
};
struct LConvInB {  // B[m][k] = im2col(in)[m][k], column Ci*9 = 1 (bias)
    const float* x;
    ConvShape s;
    struct St {
        Tap t;
        bool ok, bias;
    };
    __device__ St prep(int k) const { return St{tap_of(k), k <= s.Ci * 9, k == s.Ci * 9}; }
    __device__ void load8(const St& r, int m0, float* v) const {
        Pix p = pix_of(m0, s.OH, s.OW);
        const int mk = s.B * s.OH * s.OW;
        for (int e = 0; e < 8; ++e) {
            const int ih = 2 * p.y - 1 + r.t.kh, iw = 2 * p.x - 1 + r.t.kw;
            const bool valid = r.ok && m0 + e < mk;
            const bool in = valid && !r.bias && ih >= 0 && ih < s.H && iw >= 0 && iw < s.W;
            v[e] = r.bias ? (valid ? 1.f : 0.f)
                          : (in ? x[(((int64_t)p.n * s.Ci + r.t.c) * s.H + ih) * s.W + iw] : 0.f);
            pix_next(p, s.OH, s.OW);
        }
    }
};
struct EWGrad {
    float* dw;
    float* db;
    int Kc;
    __device__ void operator()(int co, int k, float v) const {
        if (k < Kc) dw[(int64_t)co * Kc + k] = v;
        else if (db) db[co] = v;
    }
};

// ---- linear layers: x [B][Fin], W [Fout][Fin] ----------------------------------
struct LMat {  // A[r][c]: row-major [R][C], optional second block for columns >= C1 (concatenation)
    const float* a;
    int R, C;
    const float* a2;
    int C1, C2;
    struct St {
        int r;
        bool ok;
    };
    __device__ St prep(int r) const { return St{r, r < R}; }
    __device__ float at(int r, int c) const {
        if (a2) {
            if (c < C1) return a[(int64_t)r * C1 + c];
            if (c < C1 + C2) return a2[(int64_t)r * C2 + (c - C1)];
            return 0.f;
        }
        return c < C ? a[(int64_t)r * C + c] : 0.f;
    }
    __device__ void load8(const St& st, int c0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = st.ok ? at(st.r, c0 + e) : 0.f;
    }
};
struct LMatT {  // B[k][n] = W[n][k]
    const float* w;
    int N, K;
    struct St {
        const float* p;
        bool ok;
    };
    __device__ St prep(int n) const { return St{w + (int64_t)min(n, N - 1) * K, n < N}; }
    __device__ void load8(const St& r, int k0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = (r.ok && k0 + e < K) ? r.p[k0 + e] : 0.f;
    }
};
struct LMatN {  // B[k][n] = W[k][n] (row-major [K][N])
    const float* w;
    int K, N;
    struct St {
        int n;
        bool ok;
    };
    __device__ St prep(int n) const { return St{n, n < N}; }
    __device__ void load8(const St& r, int k0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = (r.ok && k0 + e < K) ? w[(int64_t)(k0 + e) * N + r.n] : 0.f;
    }
};
struct LMasked {  // A[r][c] = masked dy[r][c]
    const float* dy;
    const float* out;
    int R, C;
    struct St {
        int64_t base;
        bool ok;
    };
    __device__ St prep(int r) const { return St{(int64_t)r * C, r < R}; }
    __device__ void load8(const St& st, int c0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = (st.ok && c0 + e < C) ? dmask(dy, out, st.base + c0 + e) : 0.f;
    }
};
struct LMaskedT {  // A[o][b] = masked dy[b][o]
    const float* dy;
    const float* out;
    int Bn, F;
    struct St {
        int o;
        bool ok;
    };
    __device__ St prep(int o) const { return St{o, o < F}; }
    __device__ void load8(const St& st, int b0, float* v) const {
        for (int e = 0; e < 8; ++e) v[e] = (st.ok && b0 + e < Bn) ? dmask(dy, out, (int64_t)(b0 + e) * F + st.o) : 0.f;
    }
};
struct LMatB {  // B[b][i] = x[b][i] (with concatenation), column Fin = 1 (bias)
    LMat x;
    int Fin;
    struct St {
        int i;
        bool ok;
    };
    __device__ St prep(int i) const { return St{i, i <= Fin}; }
    __device__ void load8(const St& st, int b0, float* v) const {
        for (int e = 0; e < 8; ++e) {
            const int b = b0 + e;
            v[e] = (!st.ok || b >= x.R) ? 0.f : (st.i == Fin ? 1.f : x.at(b, st.i));
        }
    }
};
struct EStore {
    float* y;
    const float* bias;
    int N, relu;
    __device__ void operator()(int r, int c, float v) const {
        v += bias ? bias[c] : 0.f;
        if (relu) v = fmaxf(v, 0.f);
        y[(int64_t)r * N + c] = v;
    }
};

// split-K partial sums: ws[z][row][col]
struct EPartial {
    float* ws;
    int M, N;
    __device__ void operator()(int row, int col, float v) const {
        ws[((int64_t)blockIdx.z * M + row) * N + col] = v;
    }
};

// Sum of the split-K partials in a fixed order: a workgroup takes 64
// consecutive outputs; wave q adds splits q, q + 4, ... in order, and the four
// wave sums are added in wave order.
template <class EP>
__global__ __launch_bounds__(256) void k_splitk_sum(const float* __restrict__ ws, int splits, int M, int N, EP ep) {
    __shared__ float s_part[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t mn = (int64_t)M * N;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    float v = 0.f;
    if (idx < mn)
        for (int z = q; z < splits; z += 4) v += ws[z * mn + idx];
    s_part[q][lane] = v;
    __syncthreads();
    if (q == 0 && idx < mn) ep((int)(idx / N), (int)(idx % N), ((s_part[0][lane] + s_part[1][lane]) + s_part[2][lane]) + s_part[3][lane]);
}

// Splits K when the output has too few 64x64 tiles to fill the chip and
// there is workspace (ws_floats floats) for the partial sums.
template <class LA, class LB, class EP>
hipError_t gemm(LA la, LB lb, EP ep, int M, int N, int K, hipStream_t st, float* ws = nullptr,
                size_t ws_floats = 0) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    const int gx = (M + BM - 1) / BM, gy = (N + BN - 1) / BN, tiles = gx * gy;
    const int ksteps = (K + BK - 1) / BK;
    int splits = 1;
    if (ws && tiles < 512 && ksteps >= 16) {
        splits = std::min(ksteps / 8, (1024 + tiles - 1) / tiles);
        splits = (int)std::min<size_t>((size_t)splits, ws_floats / ((size_t)M * N));
    }
    if (splits < 2) {
        hipLaunchKernelGGL((k_gemm<LA, LB, EP>), dim3(gx, gy, 1), dim3(256), 0, st, la, lb, ep, M, N, K, ksteps * BK);
        return hipGetLastError();
    }
    const int kz = ((ksteps + splits - 1) / splits) * BK;
    splits = (K + kz - 1) / kz;
    hipLaunchKernelGGL((k_gemm<LA, LB, EPartial>), dim3(gx, gy, splits), dim3(256), 0, st, la, lb,
                       EPartial{ws, M, N}, M, N, K, kz);
    const int64_t mn = (int64_t)M * N;
    hipLaunchKernelGGL((k_splitk_sum<EP>), dim3((unsigned)((mn + 63) / 64)), dim3(256), 0, st, (const float*)ws,
                       splits, M, N, ep);
    return hipGetLastError();
}

// workspace that covers every split-K GEMM gemm() sets up: at most
// ceil(1024 / tiles) splits of an M x N output with tiles = its 64x64 tiles,
// so splits * M * N <= (1024 / tiles + 1) * tiles * 4096
constexpr size_t kSplitWs = (size_t)(1024 + 512) * BM * BN;

ConvShape conv_shape(int B, int Ci, int H, int W, int Co) {
    return ConvShape{B, Ci, H, W, Co, (H + 1) / 2, (W + 1) / 2};
}

hipError_t conv_fwd(const float* x, const float* w, const float* b, float* y, ConvShape s, int relu, hipStream_t st) {
    return gemm(LConvIn{x, s}, LConvW{w, s.Co, s.Ci * 9}, EConvOut{y, b, s, relu}, s.B * s.OH * s.OW, s.Co, s.Ci * 9, st);
}
hipError_t conv_dgrad(const float* dy, const float* out, const float* w, float* dx, ConvShape s, hipStream_t st) {
    // small layers: one plain implicit GEMM fills the chip better than four
    // class GEMMs of a quarter of the rows each
    if ((int64_t)s.B * s.H * s.W < (1 << 18))
        return gemm(LConvDOut{dy, out, s}, LConvWT{w, s}, EConvDIn{dx, s}, s.B * s.H * s.W, s.Ci, s.Co * 9, st);
    for (int py = 0; py < 2; ++py)
        for (int px = 0; px < 2; ++px) {
            const DgradClass c{py, px, py ? 2 : 1, px ? 2 : 1, (s.H - py + 1) / 2, (s.W - px + 1) / 2};
            if (c.Hc <= 0 || c.Wc <= 0) continue;
            hipError_t e = gemm(LConvDOutP{dy, out, s, c}, LConvWTP{w, s, c}, EConvDInP{dx, s, c},
                                s.B * c.Hc * c.Wc, s.Ci, s.Co * c.nth * c.ntw, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}
hipError_t conv_wgrad(const float* dy, const float* out, const float* x, float* dw, float* db, ConvShape s,
                      hipStream_t st, float* ws, size_t ws_floats) {
    return gemm(LConvDOutT{dy, out, s}, LConvInB{x, s}, EWGrad{dw, db, s.Ci * 9}, s.Co, s.Ci * 9 + 1,
                s.B * s.OH * s.OW, st, ws, ws_floats);
}
hipError_t lin_fwd(LMat x, const float* w, const float* b, float* y, int Bn, int Fin, int Fout, int relu,
                   hipStream_t st) {
    return gemm(x, LMatT{w, Fout, Fin}, EStore{y, b, Fout, relu}, Bn, Fout, Fin, st);
}
hipError_t lin_dgrad(const float* dy, const float* out, const float* w, float* dx, int Bn, int Fin, int Fout,
                     hipStream_t st) {
    // dX[b][i] = sum_o dYm[b][o] W[o][i]
    return gemm(LMasked{dy, out, Bn, Fout}, LMatN{w, Fout, Fin}, EStore{dx, nullptr, Fin, 0}, Bn, Fin,
                Fout, st);
}
hipError_t lin_wgrad(const float* dy, const float* out, LMat x, float* dw, float* db, int Bn, int Fin, int Fout,
                     hipStream_t st, float* ws, size_t ws_floats) {
    return gemm(LMaskedT{dy, out, Bn, Fout}, LMatB{x, Fin}, EWGrad{dw, db, Fin}, Fout, Fin + 1, Bn, st, ws,
                ws_floats);
}

// ---- small element-wise kernels --------------------------------------------------
// dy <- dy where out > 0, else 0 (the ReLU's adjoint, applied once so that
// the layer's weight and input gradients read dy alone)
__global__ void k_relu_mask(float* __restrict__ dy, const float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(out[i] > 0.f)) dy[i] = 0.f;
}
hipError_t relu_mask(float* dy, const float* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dy, out, n);
    return hipGetLastError();
}

// Bilinear x4 upsampling of an H x W slice to a (4H) x (4W) crop, optionally
// centre-cropped / padded to 128 x 128, scaled by 1/scale.
__global__ void k_prepare(const float* __restrict__ slices, int B, int H, int W, float* __restrict__ crops) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * 128 * 128) return;
    const int x = (int)(idx % 128), y = (int)((idx / 128) % 128), b = (int)(idx / (128 * 128));
    // crop pixel -> source coordinate (centred): 4x upsampling of the slice
    const float sx = ((float)x + 0.5f) * 0.25f - 0.5f + 0.5f * (float)(W - 32);
    const float sy = ((float)y + 0.5f) * 0.25f - 0.5f + 0.5f * (float)(H - 32);
    const float fx = fminf(fmaxf(sx, 0.f), (float)(W - 1)), fy = fminf(fmaxf(sy, 0.f), (float)(H - 1));
    const int x0 = (int)floorf(fx), y0 = (int)floorf(fy);
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const float ax = fx - (float)x0, ay = fy - (float)y0;
    const float* s = slices + (int64_t)b * H * W;
    const float v = (1.f - ay) * ((1.f - ax) * s[y0 * W + x0] + ax * s[y0 * W + x1]) +
                    ay * ((1.f - ax) * s[y1 * W + x0] + ax * s[y1 * W + x1]);
    crops[idx] = v;
}

// MSE on the 6 outputs: loss = mean_b sum_c (y - t)^2 ; dy = 2 (y - t) / B
__global__ void k_mse6(const float* __restrict__ y, const float* __restrict__ t, int B, float* __restrict__ dy,
                       float* __restrict__ loss) {
    __shared__ float s[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < B * 6; i += 256) {
        const float r = y[i] - t[i];
        dy[i] = 2.f * r / (float)B;
        acc += r * r;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = s[0] / (float)B;
}

// Runs f(ws) with a stream-ordered split-K workspace (for the stand-alone
// layer entry points; the network owns its workspace).
template <class F>
int with_split_ws(hipStream_t st, F&& f) {
    float* ws = nullptr;
    if (hipMallocAsync((void**)&ws, kSplitWs * sizeof(float), st) != hipSuccess) return SVR_ERR_HIP;
    const hipError_t e = f(ws);
    const hipError_t e2 = hipFreeAsync(ws, st);
    return (e == hipSuccess && e2 == hipSuccess) ? SVR_OK : SVR_ERR_HIP;
}

}  // namespace
}  // namespace svr

using namespace svr;

// ---------------------------------------------------------------------------
struct svr_posenet {
    int device;
    hipStream_t stream;
    int max_batch;
    std::vector<int64_t> off;  // parameter offsets: conv w/b x6, fc1 w/b, fc2 w/b
    int64_t n_params = 0;
    float* params = nullptr;
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int64_t step = 0;
    float* act[7] = {};      // a0 (input view), a1..a6
    float* dact[7] = {};
    float* h = nullptr;      // fc1 output [B,256]
    float* dh = nullptr;
    float* y = nullptr;      // [B,6]
    float* dy = nullptr;
    float* dfeat = nullptr;  // [B,524]
    float* ws = nullptr;     // split-K partial sums, kSplitWs floats
};

namespace {
const int kCh[7] = {1, 32, 32, 64, 64, 128, 128};
const int kSide[7] = {128, 64, 32, 16, 8, 4, 2};
constexpr int kFeat = 128 * 2 * 2, kOrient = 12, kHidden = 256, kOut = 6;

hipError_t net_forward(svr_posenet* net, const float* crops, const float* orient, int B) {
    hipStream_t st = net->stream;
    const float* x = crops;
    for (int l = 0; l < 6; ++l) {
        ConvShape s = conv_shape(B, kCh[l], kSide[l], kSide[l], kCh[l + 1]);
        hipError_t e = conv_fwd(x, net->params + net->off[2 * l], net->params + net->off[2 * l + 1], net->act[l + 1],
                                s, 1, st);
        if (e != hipSuccess) return e;
        x = net->act[l + 1];
    }
    LMat feat{net->act[6], B, kFeat + kOrient, orient, kFeat, kOrient};
    hipError_t e = lin_fwd(feat, net->params + net->off[12], net->params + net->off[13], net->h, B, kFeat + kOrient,
                           kHidden, 1, st);
    if (e != hipSuccess) return e;
    return lin_fwd(LMat{net->h, B, kHidden, nullptr, 0, 0}, net->params + net->off[14], net->params + net->off[15],
                   net->y, B, kHidden, kOut, 0, st);
}

hipError_t net_backward(svr_posenet* net, const float* crops, const float* orient, int B) {
    hipStream_t st = net->stream;
    float* g = net->grads;
    hipError_t e;
    // fc2 (no activation on y)
    e = lin_wgrad(net->dy, nullptr, LMat{net->h, B, kHidden, nullptr, 0, 0}, g + net->off[14], g + net->off[15], B,
                  kHidden, kOut, st, net->ws, kSplitWs);
    if (e != hipSuccess) return e;
    e = lin_dgrad(net->dy, nullptr, net->params + net->off[14], net->dh, B, kHidden, kOut, st);
    if (e != hipSuccess) return e;
    // fc1 (ReLU on h)
    LMat feat{net->act[6], B, kFeat + kOrient, orient, kFeat, kOrient};
    e = relu_mask(net->dh, net->h, (int64_t)B * kHidden, st);
    if (e != hipSuccess) return e;
    e = lin_wgrad(net->dh, nullptr, feat, g + net->off[12], g + net->off[13], B, kFeat + kOrient, kHidden, st,
                  net->ws, kSplitWs);
    if (e != hipSuccess) return e;
    e = lin_dgrad(net->dh, nullptr, net->params + net->off[12], net->dfeat, B, kFeat + kOrient, kHidden, st);
    if (e != hipSuccess) return e;
    // the first 512 feature gradients (row stride 524) are d a6 ([B,128,2,2] flattened)
    e = hipMemcpy2DAsync(net->dact[6], sizeof(float) * kFeat, net->dfeat, sizeof(float) * (kFeat + kOrient),
                         sizeof(float) * kFeat, B, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    for (int l = 5; l >= 0; --l) {
        ConvShape s = conv_shape(B, kCh[l], kSide[l], kSide[l], kCh[l + 1]);
        const float* in = l == 0 ? crops : net->act[l];
        e = relu_mask(net->dact[l + 1], net->act[l + 1], (int64_t)B * s.Co * s.OH * s.OW, st);
        if (e != hipSuccess) return e;
        e = conv_wgrad(net->dact[l + 1], nullptr, in, g + net->off[2 * l], g + net->off[2 * l + 1], s, st, net->ws,
                       kSplitWs);
        if (e != hipSuccess) return e;
        if (l > 0) {
            e = conv_dgrad(net->dact[l + 1], nullptr, net->params + net->off[2 * l], net->dact[l], s, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}
}  // namespace

extern "C" {

int svr_posenet_create(svr_posenet** out, int device, void* stream, uint64_t seed, int max_batch) {
    if (!out || max_batch < 1 || max_batch > 65536) return SVR_ERR_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SVR_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return SVR_ERR_HIP;
    svr_posenet* net = new (std::nothrow) svr_posenet();
    if (!net) return SVR_ERR_CAPACITY;
    net->device = device;
    net->stream = (hipStream_t)stream;
    net->max_batch = max_batch;
    int64_t o = 0;
    std::vector<int64_t> fan;
    for (int l = 0; l < 6; ++l) {
        net->off.push_back(o);
        o += (int64_t)kCh[l + 1] * kCh[l] * 9;
        fan.push_back(kCh[l] * 9);
        net->off.push_back(o);
        o += kCh[l + 1];
        fan.push_back(0);
    }
    net->off.push_back(o); o += (int64_t)kHidden * (kFeat + kOrient); fan.push_back(kFeat + kOrient);
    net->off.push_back(o); o += kHidden; fan.push_back(0);
    net->off.push_back(o); o += (int64_t)kOut * kHidden; fan.push_back(kHidden);
    net->off.push_back(o); o += kOut; fan.push_back(0);
    net->off.push_back(o);
    net->n_params = o;
    std::vector<float> h((size_t)o, 0.f);
    std::mt19937_64 rng(seed);
    for (size_t t = 0; t + 1 < net->off.size(); ++t) {
        if (fan[t] == 0) continue;  // biases start at 0
        const double sd = (t == 14) ? 0.01 : sqrt(2.0 / fan[t]);   // He init; small last layer
        std::normal_distribution<double> nd(0.0, sd);
        for (int64_t k = net->off[t]; k < net->off[t + 1]; ++k) h[(size_t)k] = (float)nd(rng);
    }
    bool ok = hipMalloc((void**)&net->params, o * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&net->grads, o * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&net->m, o * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&net->v, o * sizeof(float)) == hipSuccess;
    for (int l = 1; l <= 6 && ok; ++l) {
        const size_t sz = (size_t)max_batch * kCh[l] * kSide[l] * kSide[l] * sizeof(float);
        ok = hipMalloc((void**)&net->act[l], sz) == hipSuccess && hipMalloc((void**)&net->dact[l], sz) == hipSuccess;
    }
    ok = ok && hipMalloc((void**)&net->h, (size_t)max_batch * kHidden * 4) == hipSuccess &&
         hipMalloc((void**)&net->dh, (size_t)max_batch * kHidden * 4) == hipSuccess &&
         hipMalloc((void**)&net->y, (size_t)max_batch * kOut * 4) == hipSuccess &&
         hipMalloc((void**)&net->dy, (size_t)max_batch * kOut * 4) == hipSuccess &&
         hipMalloc((void**)&net->dfeat, (size_t)max_batch * (kFeat + kOrient) * 4) == hipSuccess &&
         hipMalloc((void**)&net->ws, kSplitWs * sizeof(float)) == hipSuccess;
    ok = ok && hipMemcpy(net->params, h.data(), o * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(net->m, 0, o * sizeof(float)) == hipSuccess && hipMemset(net->v, 0, o * sizeof(float)) == hipSuccess;
    if (!ok) {
        svr_posenet_destroy(net);
        return SVR_ERR_HIP;
    }
    *out = net;
    return SVR_OK;
}

int svr_posenet_destroy(svr_posenet* net) {
    if (!net) return SVR_OK;
    (void)hipSetDevice(net->device);
    (void)hipStreamSynchronize(net->stream);
    float* bufs[] = {net->params, net->grads, net->m, net->v, net->h, net->dh, net->y, net->dy, net->dfeat, net->ws};
    for (float* b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 1; l <= 6; ++l) {
        if (net->act[l]) (void)hipFree(net->act[l]);
        if (net->dact[l]) (void)hipFree(net->dact[l]);
    }
    delete net;
    return SVR_OK;
}

int64_t svr_posenet_num_params(const svr_posenet* net) { return net ? net->n_params : 0; }

int svr_posenet_get_params(svr_posenet* net, float* host_out) {
    if (!net || !host_out) return SVR_ERR_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    if (hipMemcpyAsync(host_out, net->params, net->n_params * 4, hipMemcpyDeviceToHost, net->stream) != hipSuccess ||
        hipStreamSynchronize(net->stream) != hipSuccess)
        return SVR_ERR_HIP;
    return SVR_OK;
}

int svr_posenet_set_params(svr_posenet* net, const float* host_in) {
    if (!net || !host_in) return SVR_ERR_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    if (hipMemcpyAsync(net->params, host_in, net->n_params * 4, hipMemcpyHostToDevice, net->stream) != hipSuccess ||
        hipStreamSynchronize(net->stream) != hipSuccess)
        return SVR_ERR_HIP;
    return SVR_OK;
}

int svr_posenet_prepare(svr_posenet* net, const float* slices, int B, int H, int W, float* crops) {
    if (!net || !slices || !crops || B < 0 || H < 1 || W < 1) return SVR_ERR_ARG;
    if (B == 0) return SVR_OK;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    const int64_t n = (int64_t)B * 128 * 128;
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, net->stream, slices, B, H, W, crops);
    return hipGetLastError() == hipSuccess ? SVR_OK : SVR_ERR_HIP;
}

int svr_posenet_forward(svr_posenet* net, const float* crops, const float* orient, int B, float* out) {
    if (!net || !crops || !orient || !out || B < 1 || B > net->max_batch) return SVR_ERR_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    if (net_forward(net, crops, orient, B) != hipSuccess) return SVR_ERR_HIP;
    if (hipMemcpyAsync(out, net->y, (size_t)B * kOut * 4, hipMemcpyDeviceToDevice, net->stream) != hipSuccess)
        return SVR_ERR_HIP;
    return SVR_OK;
}

int svr_posenet_train_step(svr_posenet* net, const float* crops, const float* orient, const float* target, int B,
                           float lr, float* loss) {
    if (!net || !crops || !orient || !target || B < 1 || B > net->max_batch || !(lr > 0.f)) return SVR_ERR_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    if (net_forward(net, crops, orient, B) != hipSuccess) return SVR_ERR_HIP;
    hipLaunchKernelGGL(k_mse6, dim3(1), dim3(256), 0, net->stream, (const float*)net->y, target, B, net->dy, loss);
    if (hipGetLastError() != hipSuccess) return SVR_ERR_HIP;
    if (net_backward(net, crops, orient, B) != hipSuccess) return SVR_ERR_HIP;
    AdamSeg seg;
    seg.p = net->params;
    seg.g = net->grads;
    seg.n = net->n_params;
    seg.state_off = 0;
    seg.lr_a = seg.lr_b = lr;
    seg.pose_layout = 0;
    net->step += 1;
    if (launch_adam(&seg, 1, net->m, net->v, 0.9, 0.999, 1e-8, 0.0, net->step, net->stream) != hipSuccess)
        return SVR_ERR_HIP;
    return SVR_OK;
}

int svr_posenet_grads(svr_posenet* net, const float* crops, const float* orient, const float* target, int B,
                      float* loss, float* grads_out) {
    if (!net || !crops || !orient || !target || !grads_out || B < 1 || B > net->max_batch) return SVR_ERR_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SVR_ERR_HIP;
    if (net_forward(net, crops, orient, B) != hipSuccess) return SVR_ERR_HIP;
    hipLaunchKernelGGL(k_mse6, dim3(1), dim3(256), 0, net->stream, (const float*)net->y, target, B, net->dy, loss);
    if (hipGetLastError() != hipSuccess) return SVR_ERR_HIP;
    if (net_backward(net, crops, orient, B) != hipSuccess) return SVR_ERR_HIP;
    if (hipMemcpyAsync(grads_out, net->grads, net->n_params * 4, hipMemcpyDeviceToDevice, net->stream) != hipSuccess)
        return SVR_ERR_HIP;
    return SVR_OK;
}

// ---- layer primitives (DEVICE pointers, caller's stream) -------------------------
int svr_conv3x3s2_forward(void* stream, const float* x, const float* w, const float* b, float* y, int B, int Ci,
                          int H, int W, int Co, int relu) {
    if (!x || !w || !y || B < 1 || Ci < 1 || H < 1 || W < 1 || Co < 1) return SVR_ERR_ARG;
    return conv_fwd(x, w, b, y, conv_shape(B, Ci, H, W, Co), relu, (hipStream_t)stream) == hipSuccess ? SVR_OK
                                                                                                      : SVR_ERR_HIP;
}

int svr_conv3x3s2_dgrad(void* stream, const float* dy, const float* y, const float* w, float* dx, int B, int Ci,
                        int H, int W, int Co) {
    if (!dy || !w || !dx || B < 1 || Ci < 1 || H < 1 || W < 1 || Co < 1) return SVR_ERR_ARG;
    return conv_dgrad(dy, y, w, dx, conv_shape(B, Ci, H, W, Co), (hipStream_t)stream) == hipSuccess ? SVR_OK
                                                                                                   : SVR_ERR_HIP;
}

int svr_conv3x3s2_wgrad(void* stream, const float* dy, const float* y, const float* x, float* dw, float* db, int B,
                        int Ci, int H, int W, int Co) {
    if (!dy || !x || !dw || B < 1 || Ci < 1 || H < 1 || W < 1 || Co < 1) return SVR_ERR_ARG;
    return with_split_ws((hipStream_t)stream, [&](float* ws) {
        return conv_wgrad(dy, y, x, dw, db, conv_shape(B, Ci, H, W, Co), (hipStream_t)stream, ws, kSplitWs);
    });
}

int svr_linear_forward(void* stream, const float* x, const float* w, const float* b, float* y, int B, int Fin,
                       int Fout, int relu) {
    if (!x || !w || !y || B < 1 || Fin < 1 || Fout < 1) return SVR_ERR_ARG;
    return lin_fwd(LMat{x, B, Fin, nullptr, 0, 0}, w, b, y, B, Fin, Fout, relu, (hipStream_t)stream) == hipSuccess
               ? SVR_OK
               : SVR_ERR_HIP;
}

int svr_linear_dgrad(void* stream, const float* dy, const float* y, const float* w, float* dx, int B, int Fin,
                     int Fout) {
    if (!dy || !w || !dx || B < 1 || Fin < 1 || Fout < 1) return SVR_ERR_ARG;
    return lin_dgrad(dy, y, w, dx, B, Fin, Fout, (hipStream_t)stream) == hipSuccess ? SVR_OK : SVR_ERR_HIP;
}

int svr_linear_wgrad(void* stream, const float* dy, const float* y, const float* x, float* dw, float* db, int B,
                     int Fin, int Fout) {
    if (!dy || !x || !dw || B < 1 || Fin < 1 || Fout < 1) return SVR_ERR_ARG;
    return with_split_ws((hipStream_t)stream, [&](float* ws) {
        return lin_wgrad(dy, y, LMat{x, B, Fin, nullptr, 0, 0}, dw, db, B, Fin, Fout, (hipStream_t)stream, ws,
                         kSplitWs);
    });
}

}  // extern "C"
