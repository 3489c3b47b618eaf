// Slice pose, Gaussian activation, culling + projection + emission, and the
// projection adjoint.  gfx950, FP32.
//
// Geometry of one (slice i, Gaussian j) pair in the slice frame (paper Sec. 2.3,
// Eq. 4 rotated into slice coordinates):
//   m  = R_i^T (mu_j - t_i)                      Gaussian centre in the slice frame
//   S' = R_i^T Sigma_j R_i + diag(sigma_PSF^2)   observed covariance in the slice frame
// With S' = [[C0, b], [b^T, s]] (C0 the in-plane 2x2 block, s the normal entry),
// the quadratic form at the in-plane point u (third coordinate 0) splits into
//   q(u) = beta + (u - u*)^T A (u - u*),   beta = m_z^2 / s,
//   u* = m_xy - b m_z / s,  A = C^-1,  C = C0 - b b^T / s   (Schur complement),
// and det S' = det C * s.  The pair contributes inside the T-sigma footprint only
// if beta <= T^2 (plane test), then on the ellipse (u-u*)^T A (u-u*) <= T^2 - beta,
// whose bounding box has half-widths sqrt((T^2-beta) C_xx), sqrt((T^2-beta) C_yy).
// The amplitude is c_j sqrt(det Sigma_j / det S') = c_j exp(sum log s_j) / sqrt(det C s).
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kBlock = 256;
constexpr int kList = 32;

struct GAct {
    float mu[3];
    float R[9];
    float s2[3];
    float S[6];  // xx, xy, xz, yy, yz, zz
    float lsum;
    float qn[4];
    float qinv;
    float c;
};

__device__ inline float sym(const float* S, int a, int b) {
    // index into (xx, xy, xz, yy, yz, zz)
    const int idx[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    return S[idx[3 * a + b]];
}

__device__ inline void activate(const ProjectArgs& a, int64_t j, GAct& g) {
    for (int k = 0; k < 3; ++k) g.mu[k] = a.mean[3 * j + k];
    float w = a.quat[4 * j], x = a.quat[4 * j + 1], y = a.quat[4 * j + 2], z = a.quat[4 * j + 3];
    float qinv = rsqrtf(w * w + x * x + y * y + z * z);
    w *= qinv; x *= qinv; y *= qinv; z *= qinv;
    g.qn[0] = w; g.qn[1] = x; g.qn[2] = y; g.qn[3] = z;
    g.qinv = qinv;
    // R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]_x
    const float d = w * w - x * x - y * y - z * z;
    g.R[0] = d + 2 * x * x; g.R[1] = 2 * (x * y - w * z); g.R[2] = 2 * (x * z + w * y);
    g.R[3] = 2 * (x * y + w * z); g.R[4] = d + 2 * y * y; g.R[5] = 2 * (y * z - w * x);
    g.R[6] = 2 * (x * z - w * y); g.R[7] = 2 * (y * z + w * x); g.R[8] = d + 2 * z * z;
    float ls0 = a.log_scale[3 * j], ls1 = a.log_scale[3 * j + 1], ls2 = a.log_scale[3 * j + 2];
    g.s2[0] = expf(2.f * ls0); g.s2[1] = expf(2.f * ls1); g.s2[2] = expf(2.f * ls2);
    g.lsum = ls0 + ls1 + ls2;
    // Sigma = R diag(s2) R^T
    int o = 0;
    for (int p = 0; p < 3; ++p)
        for (int q = p; q < 3; ++q) {
            g.S[o++] = g.R[3 * p] * g.s2[0] * g.R[3 * q] + g.R[3 * p + 1] * g.s2[1] * g.R[3 * q + 1] +
                       g.R[3 * p + 2] * g.s2[2] * g.R[3 * q + 2];
        }
    g.c = a.amp[j];
}

__device__ inline void activate_dummy(GAct& g) {
    for (int k = 0; k < 3; ++k) { g.mu[k] = 0.f; g.s2[k] = 1.f; }
    for (int k = 0; k < 9; ++k) g.R[k] = (k % 4 == 0) ? 1.f : 0.f;
    g.S[0] = 1.f; g.S[1] = 0.f; g.S[2] = 0.f; g.S[3] = 1.f; g.S[4] = 0.f; g.S[5] = 1.f;
    g.lsum = 0.f; g.qn[0] = 1.f; g.qn[1] = g.qn[2] = g.qn[3] = 0.f; g.qinv = 1.f; g.c = 0.f;
}

// Cheap plane test: beta = m_z^2 / s_zz <= T^2.
// S = (S00, S01, S02, S11, S12, S22); the plane's coefficients turn m_z and
// S'_zz into three and six multiply-adds.
__device__ inline bool plane_pass(const GAct& g, const SlicePlane& pl, float tau2) {
    const float mz = fmaf(pl.n[2], g.mu[2], fmaf(pl.n[1], g.mu[1], pl.n[0] * g.mu[0])) - pl.d;
    float szz = fmaf(g.S[4], pl.q[5], pl.sig2z);
    szz = fmaf(g.S[2], pl.q[4], szz);
    szz = fmaf(g.S[1], pl.q[3], szz);
    szz = fmaf(g.S[5], pl.q[2], szz);
    szz = fmaf(g.S[3], pl.q[1], szz);
    szz = fmaf(g.S[0], pl.q[0], szz);
    return mz * mz <= tau2 * szz;
}

struct Proj {
    float w[3];     // mu - t (world)
    float m[3];     // slice-frame centre
    float s00, s01, s11, s02, s12, s22;  // S' entries (slice frame, incl. PSF)
    float C00, C01, C11, detC;
    float A00, A01, A11;
    float u0, u1;   // in-plane centre u* (mm)
    float beta;
    float f;        // amplitude / c
    bool keep;
};

__device__ inline void project(const GAct& g, const SlicePose& sp, const float* sig2, float tau2,
                               Proj& p) {
    p.w[0] = g.mu[0] - sp.t[0]; p.w[1] = g.mu[1] - sp.t[1]; p.w[2] = g.mu[2] - sp.t[2];
    float Sr[3][3];  // Sigma_j r_b for slice axis b (column b of R)
    for (int b = 0; b < 3; ++b) {
        const float r0 = sp.R[b], r1 = sp.R[3 + b], r2 = sp.R[6 + b];
        p.m[b] = r0 * p.w[0] + r1 * p.w[1] + r2 * p.w[2];
        Sr[b][0] = g.S[0] * r0 + g.S[1] * r1 + g.S[2] * r2;
        Sr[b][1] = g.S[1] * r0 + g.S[3] * r1 + g.S[4] * r2;
        Sr[b][2] = g.S[2] * r0 + g.S[4] * r1 + g.S[5] * r2;
    }
    auto dotc = [&](int a, int b) {
        return sp.R[a] * Sr[b][0] + sp.R[3 + a] * Sr[b][1] + sp.R[6 + a] * Sr[b][2];
    };
    p.s00 = dotc(0, 0) + sig2[0];
    p.s01 = dotc(0, 1);
    p.s11 = dotc(1, 1) + sig2[1];
    p.s02 = dotc(0, 2);
    p.s12 = dotc(1, 2);
    p.s22 = dotc(2, 2) + sig2[2];
    const float is = 1.f / p.s22;
    p.beta = p.m[2] * p.m[2] * is;
    p.C00 = p.s00 - p.s02 * p.s02 * is;
    p.C01 = p.s01 - p.s02 * p.s12 * is;
    p.C11 = p.s11 - p.s12 * p.s12 * is;
    p.detC = p.C00 * p.C11 - p.C01 * p.C01;
    const float id = 1.f / p.detC;
    p.A00 = p.C11 * id;
    p.A01 = -p.C01 * id;
    p.A11 = p.C00 * id;
    p.u0 = p.m[0] - p.s02 * p.m[2] * is;
    p.u1 = p.m[1] - p.s12 * p.m[2] * is;
    p.f = expf(g.lsum) * rsqrtf(p.detC * p.s22);
    p.keep = (p.beta <= tau2) && (p.detC > 0.f) && (p.s22 > 0.f);
}

struct Box {
    int kx0, kx1, ky0, ky1;
    bool nonempty;
};

// Shape class of an instance's clipped footprint box (h rows, w columns,
// each capped at 8): (min(h, 8) - 1) * 8 + min(w, 8) - 1.  It forms the low
// bits of the sort key, so that each tile's instances come out grouped by box
// shape and a wave of the record-per-lane tile kernels, whose lanes take
// consecutive instances, walks boxes of one shape.
__device__ inline uint32_t shape_class(int w, int h) {
    return (uint32_t)((min(h, 8) - 1) * 8 + (min(w, 8) - 1));
}

// Pixel bounding box of the footprint ellipse on slice `sg`.
__device__ inline Box pixel_box(const Proj& p, const SliceGeo& sg, float tau2) {
    Box bx;
    const float r2 = fmaxf(tau2 - p.beta, 0.f);
    const float px = p.u0 / sg.dx + 0.5f * (float)(sg.W - 1);
    const float py = p.u1 / sg.dy + 0.5f * (float)(sg.H - 1);
    const float hx = sqrtf(r2 * p.C00) / sg.dx + 1e-3f;
    const float hy = sqrtf(r2 * p.C11) / sg.dy + 1e-3f;
    const float fx0 = fmaxf(ceilf(px - hx), 0.f), fx1 = fminf(floorf(px + hx), (float)(sg.W - 1));
    const float fy0 = fmaxf(ceilf(py - hy), 0.f), fy1 = fminf(floorf(py + hy), (float)(sg.H - 1));
    bx.nonempty = p.keep && (fx0 <= fx1) && (fy0 <= fy1);
    bx.kx0 = bx.nonempty ? (int)fx0 : 0;
    bx.kx1 = bx.nonempty ? (int)fx1 : -1;
    bx.ky0 = bx.nonempty ? (int)fy0 : 0;
    bx.ky1 = bx.nonempty ? (int)fy1 : -1;
    return bx;
}

// A record that contributes nothing (slice -1, zero amplitude, no instances).
__device__ inline Record null_record() {
    Record z;
    z.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
    z.r1 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
    return z;
}

__device__ inline Record make_record(const Proj& p, const SliceGeo& sg, float c, int32_t slice) {
    Record r;
    r.r0.x = p.u0 / sg.dx + 0.5f * (float)(sg.W - 1);
    r.r0.y = p.u1 / sg.dy + 0.5f * (float)(sg.H - 1);
    r.r0.z = SVR_KZ * p.beta;
    r.r0.w = c * p.f;
    r.r1.x = SVR_KZ * p.A00 * sg.dx * sg.dx;
    r.r1.y = SVR_KZ * p.A01 * sg.dx * sg.dy;
    r.r1.z = SVR_KZ * p.A11 * sg.dy * sg.dy;
    r.r1.w = __int_as_float(slice);
    return r;
}

// ---------------------------------------------------------------------------
// K2: slice pose.  R = Exp(omega) R0 (Rodrigues), t = t0 + tau.
// ---------------------------------------------------------------------------
__global__ void k_slice_pose(const SliceGeo* __restrict__ geo, const float* __restrict__ pose,
                             SlicePose* __restrict__ out, SlicePlane* __restrict__ plane, int32_t m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float wx = pose[6 * i], wy = pose[6 * i + 1], wz = pose[6 * i + 2];
    const float th2 = wx * wx + wy * wy + wz * wz;
    const float th = sqrtf(th2);
    float A, B;
    if (th < 1e-3f) {
        A = 1.f - th2 * (1.f / 6.f);
        B = 0.5f - th2 * (1.f / 24.f);
    } else {
        const float sh = sinf(0.5f * th);
        A = sinf(th) / th;
        B = 2.f * sh * sh / th2;
    }
    // E = I + A K + B K^2, K = [w]_x ; K^2 = w w^T - th2 I
    float E[9];
    E[0] = 1.f + B * (wx * wx - th2); E[1] = -A * wz + B * wx * wy;     E[2] = A * wy + B * wx * wz;
    E[3] = A * wz + B * wx * wy;      E[4] = 1.f + B * (wy * wy - th2); E[5] = -A * wx + B * wy * wz;
    E[6] = -A * wy + B * wx * wz;     E[7] = A * wx + B * wy * wz;      E[8] = 1.f + B * (wz * wz - th2);
    const SliceGeo& g = geo[i];
    SlicePose sp;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            sp.R[3 * a + b] = E[3 * a] * g.R0[b] + E[3 * a + 1] * g.R0[3 + b] + E[3 * a + 2] * g.R0[6 + b];
    for (int k = 0; k < 3; ++k) sp.t[k] = g.t0[k] + pose[6 * i + 3 + k];
    sp.w[0] = wx;
    sp.w[1] = wy;
    sp.w[2] = wz;
    sp.pad = 0.f;
    out[i] = sp;
    if (plane) {
        SlicePlane pl;
        const float n0 = sp.R[2], n1 = sp.R[5], n2 = sp.R[8];
        pl.n[0] = n0;
        pl.n[1] = n1;
        pl.n[2] = n2;
        pl.d = fmaf(n2, sp.t[2], fmaf(n1, sp.t[1], n0 * sp.t[0]));
        pl.q[0] = n0 * n0;
        pl.q[1] = n1 * n1;
        pl.q[2] = n2 * n2;
        pl.q[3] = 2.f * n0 * n1;
        pl.q[4] = 2.f * n0 * n2;
        pl.q[5] = 2.f * n1 * n2;
        pl.sig2z = g.sig2[2];
        pl.pad = 0.f;
        plane[i] = pl;
    }
}

// ---------------------------------------------------------------------------
// K3 / K5: one thread per Gaussian, a uniform loop over the subject's slices
// doing the cheap plane test; survivors are queued in LDS and projected in
// dense bursts so that the expensive projection is not paid per slice by the
// whole wave.
// ---------------------------------------------------------------------------
template <bool kEmit>
__global__ __launch_bounds__(kBlock) void k_cull(ProjectArgs a, int2* __restrict__ counts,
                                                 const int2* __restrict__ offsets,
                                                 Record* __restrict__ rec, int2* __restrict__ rec_inst,
                                                 uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals, const int* __restrict__ only,
                                                 const int* __restrict__ overflow) {
    __shared__ uint16_t s_list[kList][kBlock];
    if (kEmit && only && only[blockIdx.x] == 0) return;  // emitted by the coalesced path
    if (kEmit && overflow && *overflow) return;          // fixed capacity exceeded: nothing is written
    const GaussBlock blk = a.blocks[blockIdx.x];
    const SubjectInfo si = a.subj[blk.subject];
    const int64_t j = blk.g_begin + threadIdx.x;
    const bool valid = j < blk.g_end;
    GAct g;
    if (valid) activate(a, j, g); else activate_dummy(g);
    const float tau2 = a.tau * a.tau;
    int cnt = 0;
    int nrec = 0, ninst = 0;
    int64_t ro = 0, io = 0;
    int2 cap = make_int2(0, 0);
    if (kEmit && valid) {
        ro = offsets[j].x;
        io = offsets[j].y;
        cap = counts[j];
    }
    const int T = a.tile;

    auto flush = [&]() {
        for (int k = 0; k < cnt; ++k) {
            const int i = si.s_begin + (int)s_list[k][threadIdx.x];
            const SliceGeo& sg = a.geo[i];
            const SlicePose& sp = a.pose[i];
            Proj p;
            project(g, sp, sg.sig2, tau2, p);
            const Box bx = pixel_box(p, sg, tau2);
            if (!kEmit) {  // count pass: no branch around the counters
                nrec += 1;
                ninst += bx.nonempty ? (bx.kx1 / T - bx.kx0 / T + 1) * (bx.ky1 / T - bx.ky0 / T + 1) : 0;
                continue;
            }
            if (!bx.nonempty) {
                // the plane crosses the footprint outside the slice: a null record
                if (kEmit && nrec < cap.x) {
                    rec[ro + nrec] = null_record();
                    rec_inst[ro + nrec] = make_int2(0, 0);
                }
                ++nrec;
                continue;
            }
            const int tx0 = bx.kx0 / T, tx1 = bx.kx1 / T, ty0 = bx.ky0 / T, ty1 = bx.ky1 / T;
            const int nt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
            if (kEmit) {
                // write only inside the slots the count pass reserved
                if (nrec >= cap.x || ninst + nt > cap.y) continue;
                const int64_t r = ro + nrec;
                rec[r] = make_record(p, sg, g.c, i);
                rec_inst[r] = make_int2((int)(io + ninst), nt);
                int64_t o = io + ninst;
                for (int ty = ty0; ty <= ty1; ++ty) {
                    const int ch = min(bx.ky1, ty * T + T - 1) - max(bx.ky0, ty * T) + 1;
                    for (int tx = tx0; tx <= tx1; ++tx) {
                        const int cw = min(bx.kx1, tx * T + T - 1) - max(bx.kx0, tx * T) + 1;
                        keys[o] = ((uint32_t)(sg.tile_base + ty * sg.ntx + tx) << kClassBits) |
                                  shape_class(cw, ch);
                        vals[o] = (uint32_t)r;
                        ++o;
                    }
                }
            }
            ++nrec;
            ninst += nt;
        }
        cnt = 0;
    };

    uint32_t word = 0;
    for (int i = si.s_begin; i < si.s_end; ++i) {
        const int li = i - si.s_begin;
        if (valid && plane_pass(g, a.plane[i], tau2)) {
            s_list[cnt][threadIdx.x] = (uint16_t)li;
            ++cnt;
            word |= 1u << (li & 31);
        }
        if (!kEmit && valid && ((li & 31) == 31 || i == si.s_end - 1)) {
            a.smask[j * a.smask_words + (li >> 5)] = word;
            word = 0;
        }
        if (__any(cnt == kList)) flush();
    }
    flush();
    if (!kEmit && valid) counts[j] = make_int2(nrec, ninst);
    if (kEmit && valid) {
        // pad reserved slots the emit pass did not fill (only if the two passes
        // ever disagreed): records with slice -1, instances with a key above
        // every tile id, so that no later stage reads them
        for (int k = nrec; k < cap.x; ++k) {
            rec[ro + k] = null_record();
            rec_inst[ro + k] = make_int2(0, 0);
        }
        for (int k = ninst; k < cap.y; ++k) {
            keys[io + k] = 0xffffffffu;
            vals[io + k] = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// K5 (coalesced): the block's records occupy one contiguous range (Gaussian
// major, slice minor).  The uniform slice loop only runs the plane test and
// drops each survivor's (Gaussian, slice) into an LDS list at its final
// position (offsets of the count pass); then every thread of the block
// projects one list entry at a time -- dense work, no divergence on the
// survivor pattern -- and records, instance ranges and instance keys are
// written with neighbouring lanes on neighbouring addresses.  Blocks whose
// record range exceeds the LDS list fall back to the per-lane path.
// ---------------------------------------------------------------------------
constexpr int kEmitCap = 6144;  // list entries per block

__global__ __launch_bounds__(kBlock) void k_emit(ProjectArgs a, const int2* __restrict__ counts,
                                                 const int2* __restrict__ offsets, Record* __restrict__ rec,
                                                 int2* __restrict__ rec_inst, uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals, int* __restrict__ fallback,
                                                 const int* __restrict__ overflow) {
    __shared__ uint32_t s_list[kEmitCap];
    __shared__ float s_act[11][kBlock];
    __shared__ int s_wsum[kBlock / 64];
    __shared__ int s_pad_from;  // first instance slot (block-relative) left unwritten
    const GaussBlock blk = a.blocks[blockIdx.x];
    const SubjectInfo si = a.subj[blk.subject];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ng = (int)(blk.g_end - blk.g_begin);
    const int64_t R0 = offsets[blk.g_begin].x, I0 = offsets[blk.g_begin].y;
    const int64_t R1 = offsets[blk.g_end - 1].x + counts[blk.g_end - 1].x;
    const int64_t I1 = offsets[blk.g_end - 1].y + counts[blk.g_end - 1].y;
    const int nrec_blk = (int)(R1 - R0);
    if (overflow && *overflow) {  // fixed capacity exceeded: nothing is written
        if (tid == 0) fallback[blockIdx.x] = 0;
        return;
    }
    if (nrec_blk > kEmitCap) {
        if (tid == 0) fallback[blockIdx.x] = 1;
        return;
    }
    if (tid == 0) {
        fallback[blockIdx.x] = 0;
        s_pad_from = (int)(I1 - I0);
    }
    const int64_t j = blk.g_begin + tid;
    const bool valid = tid < ng;
    if (valid) {  // the block's activations, read by every survivor of the Gaussian
        GAct g;
        activate(a, j, g);
        for (int q = 0; q < 3; ++q) s_act[q][tid] = g.mu[q];
        for (int q = 0; q < 6; ++q) s_act[3 + q][tid] = g.S[q];
        s_act[9][tid] = g.lsum;
        s_act[10][tid] = g.c;
    }
    const float tau2 = a.tau * a.tau;
    int loff = 0, lcap = 0, k = 0;
    if (valid) {
        loff = (int)(offsets[j].x - R0);
        lcap = counts[j].x;
    }
    // survivors of the count pass's plane test, in slice order
    const int nwords = (si.s_end - si.s_begin + 31) >> 5;
    for (int wd = 0; wd < nwords; ++wd) {
        uint32_t m = valid ? a.smask[j * a.smask_words + wd] : 0u;
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1u;
            if (k < lcap) s_list[loff + k] = ((uint32_t)tid << 16) | (uint32_t)(wd * 32 + b);
            ++k;
        }
    }
    // slots the plane test did not fill again (only if the passes ever disagreed)
    for (int q = k; q < lcap; ++q) s_list[loff + q] = 0xffffffffu;
    __syncthreads();
    const int T = a.tile;
    int64_t ibase = I0;
    for (int t0 = 0; t0 < nrec_blk; t0 += kBlock) {
        const int t = t0 + tid;
        const uint32_t e = (t < nrec_blk) ? s_list[t] : 0xffffffffu;
        Record R = null_record();
        Box bx;
        bx.nonempty = false;
        int nt = 0, sl = -1;
        int tbase = 0, ntx = 0;  // the slice's first tile and tiles per row, in registers: a load between
                                 // the instance stores below would wait for the stores too
        const SliceGeo* sgp = nullptr;
        if (e != 0xffffffffu) {
            const int jl = (int)(e >> 16);
            sl = si.s_begin + (int)(e & 0xffffu);
            GAct gj;  // the fields projection and record read
            for (int q = 0; q < 3; ++q) gj.mu[q] = s_act[q][jl];
            for (int q = 0; q < 6; ++q) gj.S[q] = s_act[3 + q][jl];
            gj.lsum = s_act[9][jl];
            gj.c = s_act[10][jl];
            sgp = &a.geo[sl];
            Proj p;
            project(gj, a.pose[sl], sgp->sig2, tau2, p);
            bx = pixel_box(p, *sgp, tau2);
            tbase = sgp->tile_base;
            ntx = sgp->ntx;
            if (bx.nonempty) {
                R = make_record(p, *sgp, gj.c, sl);
                nt = (bx.kx1 / T - bx.kx0 / T + 1) * (bx.ky1 / T - bx.ky0 / T + 1);
            }
        }
        // block exclusive scan of instance counts
        int incl = nt;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_wsum[w] = incl;
        __syncthreads();
        int wbase = 0, tot = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            if (q < w) wbase += s_wsum[q];
            tot += s_wsum[q];
        }
        __syncthreads();
        int64_t o = ibase + wbase + incl - nt;
        if (nt > 0 && o + nt > I1) {  // never write past the block's reserved instances
            atomicMin(&s_pad_from, (int)(min(o, I1) - I0));
            nt = 0;
        }
        if (t < nrec_blk) {
            rec[R0 + t] = nt > 0 ? R : null_record();
            rec_inst[R0 + t] = make_int2((int)o, nt);
        }
        if (nt > 0) {
            const int tx0 = bx.kx0 / T, tx1 = bx.kx1 / T, ty0 = bx.ky0 / T, ty1 = bx.ky1 / T;
            for (int ty = ty0; ty <= ty1; ++ty) {
                const int ch = min(bx.ky1, ty * T + T - 1) - max(bx.ky0, ty * T) + 1;
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const int cw = min(bx.kx1, tx * T + T - 1) - max(bx.kx0, tx * T) + 1;
                    keys[o] = ((uint32_t)(tbase + ty * ntx + tx) << kClassBits) | shape_class(cw, ch);
                    vals[o] = (uint32_t)(R0 + t);
                    ++o;
                }
            }
        }
        ibase += tot;
    }
    // pad reserved instances nobody wrote (only if the passes ever disagreed)
    __syncthreads();
    const int64_t pad0 = min(ibase, I0 + (int64_t)s_pad_from);
    for (int64_t q = pad0 + tid; q < I1; q += kBlock) {
        keys[q] = 0xffffffffu;
        vals[q] = 0u;
    }
}

// ---------------------------------------------------------------------------
// K10: projection adjoint.  One workgroup per block of Gaussians (never
// straddling subjects); its records are contiguous (Gaussian-major emission),
// so thread k of the block takes the block's records k, k + 256, ... and all
// record, instance-slot and gradient reads are coalesced.  A record's owning
// Gaussian is found by binary search over the block's record offsets in LDS.
// Each record's gradient (sum of its instance slots, in stored units) is
// chained back through the pixel-unit scaling, the Schur complement and the
// slice rotation to
//   dL/dSigma_j (symmetric), dL/dmu_j, dL/dc_j and the direct sqrt(det) term,
// reduced over lanes of the same Gaussian with a segmented DPP scan and
// added once per segment into LDS accumulators; the slice-pose gradient
// (left perturbation delta and translation) goes to per-block LDS slice
// accumulators.  Finally thread j chains dL/dSigma_j to the log-scales and
// the quaternion and writes the Gaussian's gradient.
// ---------------------------------------------------------------------------
// The projection adjoint runs each Gaussian block as kBlock / kPartGauss
// workgroups of kPartGauss Gaussians.  Whole blocks of 256 Gaussians, at six
// resident per CU (LDS), filled the chip about 1.3 times over and left a
// tail; parts of 128 halve each workgroup's work and LDS (measured 6 %
// faster; parts of 64 were slower).
constexpr int kPartGauss = 128;
constexpr int kGAcc = 11;  // GS (6), gmu (3), gc, glsum
constexpr int kGAct = 11;  // staged activation: mu (3), Sigma (6), lsum, c

// One step of an inclusive sum over runs of equal keys across a wave (keys
// non-decreasing over lanes): lanes take the value kCtrl moves to them when
// it comes from a lane with the same key.  row_shr:n (0x110 + n) shifts
// inside 16-lane rows; row_bcast:15 (0x142, rows 1 and 3) and row_bcast:31
// (0x143, rows 2 and 3) carry a row's last lane into the following rows.
// Lanes without a source keep old = 0 (value) or -2 (key, never a real key).
template <int kCtrl, int kRowMask, int kN>
__device__ inline void seg_scan_step(float (&v)[kN], int key) {
    const int src_key = __builtin_amdgcn_update_dpp(-2, key, kCtrl, kRowMask, 0xf, false);
    const bool take = src_key == key;
    for (int q = 0; q < kN; ++q) {
        const float t = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), kCtrl, kRowMask, 0xf, false));
        v[q] += take ? t : 0.f;
    }
}

template <int kN>
__device__ inline void seg_scan(float (&v)[kN], int key) {
    seg_scan_step<0x111, 0xf>(v, key);
    seg_scan_step<0x112, 0xf>(v, key);
    seg_scan_step<0x114, 0xf>(v, key);
    seg_scan_step<0x118, 0xf>(v, key);
    seg_scan_step<0x142, 0xa>(v, key);
    seg_scan_step<0x143, 0xc>(v, key);
}

template <int NGS>
__global__ __launch_bounds__(kBlock, 7) void k_project_backward(
    ProjectArgs a, const int2* __restrict__ offsets, const int2* __restrict__ counts,
    const Record* __restrict__ rec, const int2* __restrict__ rec_inst, const float4* __restrict__ inst_grad,
    int64_t n_inst, float* __restrict__ g_mean, float* __restrict__ g_log_scale, float* __restrict__ g_quat,
    float* __restrict__ g_amp, float* __restrict__ pose_acc, int use_lds, float* __restrict__ pose_part) {
    // dynamic LDS: per-slice pose sums [6 * ns] floats, then this pass's
    // fixed-point pose sums [6 * ns] int64 (8-byte aligned: 6 * ns floats is
    // a multiple of 8 bytes)
    extern __shared__ float s_pose[];
    __shared__ float s_wmax[kBlock / 64];
    __shared__ int s_roff[NGS + 1];  // record offsets of the part's Gaussians, relative to the first
    __shared__ float s_gacc[kGAcc][NGS];
    __shared__ float s_act[kGAct][NGS];
    // workgroup = one NGS-Gaussian part of a Gaussian block
    constexpr int NS = kBlock / NGS;
    static_assert(NS == kProjParts, "parts per Gaussian block");
    const GaussBlock blk = a.blocks[blockIdx.x / NS];
    const int64_t g0 = blk.g_begin + (int64_t)(blockIdx.x % NS) * NGS;
    const SubjectInfo si = a.subj[blk.subject];
    const int ns = si.s_end - si.s_begin;
    float* const prow = pose_part + si.pose_base + (int64_t)((int)blockIdx.x - si.part0) * 6 * ns;
    if (g0 >= blk.g_end) {  // empty part (uniform): a zero row of pose sums
        if (use_lds)
            for (int k = threadIdx.x; k < 6 * ns; k += kBlock) prow[k] = 0.f;
        return;
    }
    const int64_t g1 = min(g0 + (int64_t)NGS, blk.g_end);
    unsigned long long* s_ipose = reinterpret_cast<unsigned long long*>(s_pose + 6 * ns);
    const int tid = threadIdx.x, lane = tid & 63;
    const int ng = (int)(g1 - g0);
    const int64_t R0 = offsets[g0].x;
    {
        const int64_t j = g0 + tid;
        if (tid < ng) s_roff[tid] = (int)(offsets[j].x - R0);
        if (tid == ng - 1) s_roff[ng] = (int)(offsets[j].x + counts[j].x - R0);
        if (tid < NGS)
            for (int q = 0; q < kGAcc; ++q) s_gacc[q][tid] = 0.f;
        if (tid < ng) {
            GAct g;
            activate(a, j, g);
            for (int k = 0; k < 3; ++k) s_act[k][tid] = g.mu[k];
            for (int k = 0; k < 6; ++k) s_act[3 + k][tid] = g.S[k];
            s_act[9][tid] = g.lsum;
            s_act[10][tid] = g.c;
        }
    }
    if (use_lds)
        for (int k = tid; k < 6 * ns; k += blockDim.x) {
            s_pose[k] = 0.f;
            s_ipose[k] = 0ull;
        }
    __syncthreads();
    const int nrec_blk = s_roff[ng];
    const float tau2 = a.tau * a.tau;
    for (int base = 0; base < nrec_blk; base += kBlock) {
        const int lr = base + tid;
        const bool valid = lr < nrec_blk;
        bool has_pose = false;
        int li = 0;
        float pd[6];
        // owning Gaussian: largest g with s_roff[g] <= lr
        int g = 0;
        if (valid) {
            int lo = 0, hi = ng - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_roff[mid] <= lr) lo = mid; else hi = mid - 1;
            }
            g = lo;
        }
        float acc[kGAcc];
        for (int q = 0; q < kGAcc; ++q) acc[q] = 0.f;
        // Loads in two rounds, each issued at once without branches (indices
        // clamped, results selected): the record and its instance range, then
        // the first two instance gradients (most records have one or two) and
        // the slice's geometry and pose.
        const int64_t rl = R0 + min(lr, nrec_blk - 1);
        const Record Rl = rec[rl];
        const int2 ri = rec_inst[rl];
        __builtin_amdgcn_sched_barrier(0);
        const int i = valid ? __float_as_int(Rl.r1.w) : -1;
        const bool live = valid && i >= si.s_begin && i < si.s_end;
        const int is_ = live ? i : si.s_begin;
        const int64_t e0 = ri.x, ecnt = live ? ri.y : 0;
        const int64_t ea = n_inst > 0 ? min(max(e0, (int64_t)0), n_inst - 1) : 0;
        const int64_t eb = n_inst > 0 ? min(max(e0 + 1, (int64_t)0), n_inst - 1) : 0;
        float4 u0 = make_float4(0.f, 0.f, 0.f, 0.f), w0 = u0, u1 = u0, w1 = u0;
        if (n_inst > 0) {  // uniform
            u0 = inst_grad[2 * ea];
            w0 = inst_grad[2 * ea + 1];
            u1 = inst_grad[2 * eb];
            w1 = inst_grad[2 * eb + 1];
        }
        const SlicePose sp = a.pose[is_];
        const float3 sig2 = make_float3(a.geo[is_].sig2[0], a.geo[is_].sig2[1], a.geo[is_].sig2[2]);
        const float sdx = a.geo[is_].dx, sdy = a.geo[is_].dy;
        __builtin_amdgcn_sched_barrier(0);
        if (live) {
            GAct ga;  // only the fields the projection and its adjoint read
            for (int k = 0; k < 3; ++k) ga.mu[k] = s_act[k][g];
            for (int k = 0; k < 6; ++k) ga.S[k] = s_act[3 + k][g];
            ga.lsum = s_act[9][g];
            ga.c = s_act[10][g];
            // instance sums in slot order (the first two from the loads above)
            float G[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (ecnt >= 1 && e0 >= 0 && e0 < n_inst) {
                G[0] += u0.x; G[1] += u0.y; G[2] += u0.z; G[3] += u0.w;
                G[4] += w0.x; G[5] += w0.y; G[6] += w0.z;
            }
            if (ecnt >= 2 && e0 + 1 < n_inst) {
                G[0] += u1.x; G[1] += u1.y; G[2] += u1.z; G[3] += u1.w;
                G[4] += w1.x; G[5] += w1.y; G[6] += w1.z;
            }
            for (int64_t e = e0 + 2; e < e0 + ecnt && e < n_inst; ++e) {
                const float4 u = inst_grad[2 * e], w = inst_grad[2 * e + 1];
                G[0] += u.x; G[1] += u.y; G[2] += u.z; G[3] += u.w;
                G[4] += w.x; G[5] += w.y; G[6] += w.z;
            }
            Proj p;
            const float sg2[3] = {sig2.x, sig2.y, sig2.z};
            project(ga, sp, sg2, tau2, p);
            const float is = 1.f / p.s22;
            // stored units -> natural units
            const float dbeta = SVR_KZ * G[1];
            const float du0 = G[2] / sdx, du1 = G[3] / sdy;
            const float ga00 = SVR_KZ * sdx * sdx * G[4];
            const float ga01 = 0.5f * SVR_KZ * sdx * sdy * G[5];
            const float ga11 = SVR_KZ * sdy * sdy * G[6];
            // A = C^-1  ->  G_C = -A G_A A
            const float t00 = p.A00 * ga00 + p.A01 * ga01, t01 = p.A00 * ga01 + p.A01 * ga11;
            const float t10 = p.A01 * ga00 + p.A11 * ga01, t11 = p.A01 * ga01 + p.A11 * ga11;
            float gc00 = -(t00 * p.A00 + t01 * p.A01);
            float gc01 = -(t00 * p.A01 + t01 * p.A11);
            float gc11 = -(t10 * p.A01 + t11 * p.A11);
            // amplitude a = c f, ln f = lsum - 1/2 ln det C - 1/2 ln s
            const float gam = G[0] * ga.c * p.f;
            acc[9] = G[0] * p.f;
            acc[10] = gam;
            gc00 -= 0.5f * gam * p.A00;
            gc01 -= 0.5f * gam * p.A01;
            gc11 -= 0.5f * gam * p.A11;
            float ds = -0.5f * gam * is;
            // beta = m_z^2 / s
            float dm2 = dbeta * 2.f * p.m[2] * is;
            ds -= dbeta * p.beta * is;
            // u* = m_xy - b m_z / s
            const float h = p.s02 * du0 + p.s12 * du1;
            dm2 -= h * is;
            float db0 = -du0 * p.m[2] * is, db1 = -du1 * p.m[2] * is;
            ds += h * p.m[2] * is * is;
            // C = C0 - b b^T / s
            const float Gb0 = gc00 * p.s02 + gc01 * p.s12, Gb1 = gc01 * p.s02 + gc11 * p.s12;
            db0 -= 2.f * Gb0 * is;
            db1 -= 2.f * Gb1 * is;
            ds += (p.s02 * Gb0 + p.s12 * Gb1) * is * is;
            // slice-frame gradient of S' (full-matrix, symmetric)
            const float Gp[9] = {gc00, gc01, 0.5f * db0, gc01, gc11, 0.5f * db1, 0.5f * db0, 0.5f * db1, ds};
            // world frame: G_S = R G' R^T
            float RG[9];
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v)
                    RG[3 * u + v] = sp.R[3 * u] * Gp[v] + sp.R[3 * u + 1] * Gp[3 + v] + sp.R[3 * u + 2] * Gp[6 + v];
            {
                int o = 0;
                for (int u = 0; u < 3; ++u)
                    for (int v = u; v < 3; ++v)
                        acc[o++] = RG[3 * u] * sp.R[3 * v] + RG[3 * u + 1] * sp.R[3 * v + 1] + RG[3 * u + 2] * sp.R[3 * v + 2];
            }
            // m = R^T (mu - t): dmu = R dm, dt = -R dm
            const float dm[3] = {du0, du1, dm2};
            float Rdm[3];
            for (int u = 0; u < 3; ++u) Rdm[u] = sp.R[3 * u] * dm[0] + sp.R[3 * u + 1] * dm[1] + sp.R[3 * u + 2] * dm[2];
            acc[6] = Rdm[0];
            acc[7] = Rdm[1];
            acc[8] = Rdm[2];
            // left perturbation of R_i: d delta = (R dm) x w + 2 (B12, B20, B01),
            // B = G_S Sigma_j - Sigma_j G_S
            float GSig[9];
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) {
                    float t = 0.f;
                    for (int q = 0; q < 3; ++q) t += sym(acc, u, q) * sym(ga.S, q, v);
                    GSig[3 * u + v] = t;
                }
            const float B12 = GSig[5] - GSig[7], B20 = GSig[6] - GSig[2], B01 = GSig[1] - GSig[3];
            pd[0] = Rdm[1] * p.w[2] - Rdm[2] * p.w[1] + 2.f * B12;
            pd[1] = Rdm[2] * p.w[0] - Rdm[0] * p.w[2] + 2.f * B20;
            pd[2] = Rdm[0] * p.w[1] - Rdm[1] * p.w[0] + 2.f * B01;
            pd[3] = -Rdm[0];
            pd[4] = -Rdm[1];
            pd[5] = -Rdm[2];
            if (use_lds) {
                li = i - si.s_begin;
                has_pose = true;
            } else {
                for (int q = 0; q < 6; ++q) atomicAdd(&pose_acc[6 * i + q], pd[q]);
            }
        }
        // segmented inclusive scan over lanes sharing the same Gaussian
        const int key = valid ? g : -1;
        seg_scan(acc, key);
        const int knext = __shfl_down(key, 1, 64);
        const bool tail = valid && (lane == 63 || knext != key);
        if (tail)
            for (int q = 0; q < kGAcc; ++q) atomicAdd(&s_gacc[q][g], acc[q]);
        if (use_lds) {
            // Pose sums per slice.  LDS float atomics are slow on this GPU and
            // integer ones are not, so each pass adds its values in fixed point:
            // quantum 2^(e - 40) with 2^e > the pass's largest |value|, exact
            // sums of up to 256 values below 2^49 quanta; the slice's owner
            // thread then adds the pass total to its float sum.
            float m = 0.f;
            if (has_pose)
                for (int q = 0; q < 6; ++q) m = fmaxf(m, fabsf(pd[q]));
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
            if (lane == 0) s_wmax[tid >> 6] = m;
            __syncthreads();
            m = fmaxf(fmaxf(s_wmax[0], s_wmax[1]), fmaxf(s_wmax[2], s_wmax[3]));
            if (!isfinite(m)) {  // keep a non-finite gradient visible (rare path)
                if (has_pose)
                    for (int q = 0; q < 6; ++q) atomicAdd(&s_pose[6 * li + q], pd[q]);
                m = 0.f;
                has_pose = false;
            }
            const int ex = m > 0.f ? ilogbf(m) + 1 : 0;
            const float to_q = ldexpf(1.f, 40 - ex);
            if (has_pose)
                for (int q = 0; q < 6; ++q)
                    atomicAdd(&s_ipose[6 * li + q], (unsigned long long)llrintf(pd[q] * to_q));
            __syncthreads();
            const double from_q = ldexp(1.0, ex - 40);
            for (int k = tid; k < 6 * ns; k += kBlock) {
                const long long v = (long long)s_ipose[k];
                if (v != 0) {
                    s_pose[k] += (float)((double)v * from_q);
                    s_ipose[k] = 0ull;
                }
            }
        }
    }
    __syncthreads();
    if (tid < ng) {
        const int64_t j = g0 + tid;
        GAct g;
        activate(a, j, g);
        float GS[6];
        for (int q = 0; q < 6; ++q) GS[q] = s_gacc[q][tid];
        const float glsum = s_gacc[10][tid];
        // Sigma_j = R diag(s^2) R^T
        float GR[9];  // G_S R_j
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v)
                GR[3 * u + v] = sym(GS, u, 0) * g.R[v] + sym(GS, u, 1) * g.R[3 + v] + sym(GS, u, 2) * g.R[6 + v];
        for (int k = 0; k < 3; ++k) {
            // (R^T G R)_kk = sum_u R_uk (G R)_uk
            const float d = g.R[k] * GR[k] + g.R[3 + k] * GR[3 + k] + g.R[6 + k] * GR[6 + k];
            g_log_scale[3 * j + k] = glsum + 2.f * g.s2[k] * d;
        }
        float dR[9];  // dL/dR_j = 2 G_S R_j diag(s^2)
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) dR[3 * u + v] = 2.f * GR[3 * u + v] * g.s2[v];
        // R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]_x, differentiated in (w, v)
        const float w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
        const float tr = dR[0] + dR[4] + dR[8];
        const float ax = dR[7] - dR[5], ay = dR[2] - dR[6], az = dR[3] - dR[1];
        const float sv0 = (2.f * dR[0]) * x + (dR[1] + dR[3]) * y + (dR[2] + dR[6]) * z;
        const float sv1 = (dR[1] + dR[3]) * x + (2.f * dR[4]) * y + (dR[5] + dR[7]) * z;
        const float sv2 = (dR[2] + dR[6]) * x + (dR[5] + dR[7]) * y + (2.f * dR[8]) * z;
        float gq[4];
        gq[0] = 2.f * w * tr + 2.f * (x * ax + y * ay + z * az);
        gq[1] = -2.f * x * tr + 2.f * sv0 + 2.f * w * ax;
        gq[2] = -2.f * y * tr + 2.f * sv1 + 2.f * w * ay;
        gq[3] = -2.f * z * tr + 2.f * sv2 + 2.f * w * az;
        const float dp = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
        for (int k = 0; k < 4; ++k) g_quat[4 * j + k] = (gq[k] - g.qn[k] * dp) * g.qinv;
        for (int k = 0; k < 3; ++k) g_mean[3 * j + k] = s_gacc[6 + k][tid];
        g_amp[j] = s_gacc[9][tid];
    }
    if (use_lds) {  // the part's row of pose sums, reduced over parts in a fixed order below
        __syncthreads();
        for (int k = tid; k < 6 * ns; k += blockDim.x) prow[k] = s_pose[k];
    }
}

// Pose sums, first level: work item (subject, 64 columns, kPoseRowChunk
// parts); wave q adds parts q, q + 4, ... of the item in order, the four wave
// sums are added in wave order.
__global__ __launch_bounds__(256) void k_pose_sum_parts(const float* __restrict__ part,
                                                        const SubjectInfo* __restrict__ subj,
                                                        const int4* __restrict__ w1, float* __restrict__ pp) {
    __shared__ float s_sum[4][64];
    const int4 w = w1[blockIdx.x];  // subject, column group, row chunk
    const SubjectInfo si = subj[w.x];
    const int C = 6 * (si.s_end - si.s_begin);
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = w.y * 64 + lane;
    const int p0 = w.z * kPoseRowChunk, p1 = min(si.nparts, p0 + kPoseRowChunk);
    float v = 0.f;
    if (col < C)
        for (int p = p0 + q; p < p1; p += 4) v += part[si.pose_base + (int64_t)p * C + col];
    s_sum[q][lane] = v;
    __syncthreads();
    if (q == 0 && col < C)
        pp[si.pp_base + (int64_t)w.z * C + col] = (s_sum[0][lane] + s_sum[1][lane]) + (s_sum[2][lane] + s_sum[3][lane]);
}

// Pose sums, second level: work item (subject, 64 columns); wave q adds the
// first level's rows q, q + 4, ... in order, the four wave sums are added in
// wave order -> pose_acc (overwritten).
__global__ __launch_bounds__(256) void k_pose_sum_rows(const float* __restrict__ pp,
                                                       const SubjectInfo* __restrict__ subj,
                                                       const int2* __restrict__ w2, float* __restrict__ pose_acc) {
    __shared__ float s_sum[4][64];
    const int2 w = w2[blockIdx.x];  // subject, column group
    const SubjectInfo si = subj[w.x];
    const int C = 6 * (si.s_end - si.s_begin);
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = w.y * 64 + lane;
    float v = 0.f;
    if (col < C)
        for (int r = q; r < si.nrc; r += 4) v += pp[si.pp_base + (int64_t)r * C + col];
    s_sum[q][lane] = v;
    __syncthreads();
    if (q == 0 && col < C)
        pose_acc[6 * (int64_t)si.s_begin + col] = (s_sum[0][lane] + s_sum[1][lane]) + (s_sum[2][lane] + s_sum[3][lane]);
}

// K11: d omega = J_l(omega)^T d delta, d tau = d t.
__global__ void k_pose_chain(const float* __restrict__ pose, const float* __restrict__ acc,
                             float* __restrict__ g_pose, int32_t m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float wx = pose[6 * i], wy = pose[6 * i + 1], wz = pose[6 * i + 2];
    const float th2 = wx * wx + wy * wy + wz * wz;
    const float th = sqrtf(th2);
    float B, Cc;
    if (th < 0.5f) {
        B = 0.5f - th2 * (1.f / 24.f - th2 * (1.f / 720.f));
        Cc = 1.f / 6.f - th2 * (1.f / 120.f - th2 * (1.f / 5040.f - th2 * (1.f / 362880.f)));
    } else {
        const float sh = sinf(0.5f * th);
        B = 2.f * sh * sh / th2;
        Cc = (th - sinf(th)) / (th2 * th);
    }
    // J = I + B K + C K^2, K = [w]_x, K^2 = w w^T - th2 I ; out = J^T d
    const float d0 = acc[6 * i], d1 = acc[6 * i + 1], d2 = acc[6 * i + 2];
    const float J[9] = {1.f + Cc * (wx * wx - th2), -B * wz + Cc * wx * wy, B * wy + Cc * wx * wz,
                        B * wz + Cc * wx * wy, 1.f + Cc * (wy * wy - th2), -B * wx + Cc * wy * wz,
                        -B * wy + Cc * wx * wz, B * wx + Cc * wy * wz, 1.f + Cc * (wz * wz - th2)};
    for (int a = 0; a < 3; ++a) g_pose[6 * i + a] = J[a] * d0 + J[3 + a] * d1 + J[6 + a] * d2;
    for (int a = 0; a < 3; ++a) g_pose[6 * i + 3 + a] = acc[6 * i + 3 + a];
}

}  // namespace

hipError_t launch_slice_pose(const SliceGeo* geo, const float* pose, SlicePose* out, int32_t m,
                             hipStream_t st, SlicePlane* plane) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_pose, dim3((m + 127) / 128), dim3(128), 0, st, geo, pose, out, plane, m);
    return hipGetLastError();
}

hipError_t launch_cull_count(const ProjectArgs& a, int2* counts, hipStream_t st) {
    if (a.n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cull<false>, dim3(a.n_blocks), dim3(kBlock), 0, st, a, counts,
                       (const int2*)nullptr, (Record*)nullptr, (int2*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                       (const int*)nullptr, (const int*)nullptr);
    return hipGetLastError();
}

hipError_t launch_emit(const ProjectArgs& a, const int2* counts, const int2* offsets, Record* rec,
                       int2* rec_inst, uint32_t* keys, uint32_t* vals, int* fallback, const int* overflow,
                       hipStream_t st) {
    if (a.n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3(a.n_blocks), dim3(kBlock), 0, st, a, counts, offsets, rec, rec_inst, keys, vals,
                       fallback, overflow);
    hipLaunchKernelGGL(k_cull<true>, dim3(a.n_blocks), dim3(kBlock), 0, st, a, const_cast<int2*>(counts),
                       offsets, rec, rec_inst, keys, vals, (const int*)fallback, overflow);
    return hipGetLastError();
}

hipError_t launch_project_backward(const ProjectArgs& a, const int2* offsets, const int2* counts,
                                   const Record* rec, const int2* rec_inst, const float4* inst_grad,
                                   int64_t n_inst, float* g_mean, float* g_log_scale, float* g_quat,
                                   float* g_amp, float* pose_acc, int32_t max_subject_slices, float* pose_part,
                                   float* pose_pp, const int4* w1, int32_t n_w1, const int2* w2, int32_t n_w2,
                                   int32_t m, hipStream_t st) {
    if (a.n_blocks <= 0) return hipSuccess;
    const int use_lds = (max_subject_slices <= 512 && pose_part && pose_pp && w1) ? 1 : 0;  // 72 B LDS per slice
    const size_t lds = use_lds ? (sizeof(float) + sizeof(unsigned long long)) * 6 * (size_t)max_subject_slices : 0;
    constexpr int NGS = kPartGauss;
    hipLaunchKernelGGL(k_project_backward<NGS>, dim3(a.n_blocks * (kBlock / NGS)), dim3(kBlock), lds, st, a, offsets,
                       counts, rec, rec_inst, inst_grad, n_inst, g_mean, g_log_scale, g_quat, g_amp, pose_acc,
                       use_lds, pose_part);
    if (use_lds && m > 0) {
        if (n_w1 > 0)
            hipLaunchKernelGGL(k_pose_sum_parts, dim3((unsigned)n_w1), dim3(256), 0, st, (const float*)pose_part,
                               a.subj, w1, pose_pp);
        if (n_w2 > 0)
            hipLaunchKernelGGL(k_pose_sum_rows, dim3((unsigned)n_w2), dim3(256), 0, st, (const float*)pose_pp,
                               a.subj, w2, pose_acc);
    }
    return hipGetLastError();
}

hipError_t launch_pose_chain(const float* pose, const float* pose_acc, float* g_pose, int32_t m,
                             hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_chain, dim3((m + 127) / 128), dim3(128), 0, st, pose, pose_acc, g_pose, m);
    return hipGetLastError();
}

}  // namespace svr
