// C ABI of libsvr: context, geometry, and the project_bin / forward /
// backward / step pipeline.  See include/svr.h for the contract.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "svr.h"
#include "svr_internal.h"

namespace svr {
hipError_t launch_scan_int(const int* in, int* out, int64_t n, long long* totals, void* tmp,
                           hipStream_t st);
hipError_t launch_tile_cost_keys(const int2* ranges, int32_t n_tiles, uint32_t* keys, uint32_t* vals,
                                 hipStream_t st);
}  // namespace svr

using namespace svr;

namespace {
enum Stage {
    ST_SLICE_POSE, ST_CULL_COUNT, ST_SCAN, ST_EMIT, ST_SORT, ST_TILE_RANGES, ST_TILE_ORDER, ST_MASK_SUM,
    ST_FORWARD, ST_LOSS, ST_ZERO, ST_BACKWARD, ST_PROJECT_BACKWARD, ST_POSE_CHAIN, ST_ADAM, ST_TOPK_KNN,
    ST_TOPK_INVERSE, ST_TOPK_FORWARD, ST_TOPK_BACKWARD, ST_CLASS_ORDER, ST_COUNT
};
const char* const kStageNames[ST_COUNT] = {
    "slice_pose", "cull_count", "scan", "emit", "sort", "tile_ranges", "tile_order", "mask_sum",
    "forward_tile", "loss_reduce", "zero_fill", "backward_tile", "project_backward", "pose_chain", "adam",
    "topk_knn", "topk_inverse", "topk_forward", "topk_backward", "class_order"};

constexpr int kGaussBlock = 256;
constexpr int kMaxSubjectSlices = 4096;

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;  // elements
};
}  // namespace

struct svr_ctx {
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    std::string err;
    int n_cu = 256;

    // geometry (host)
    bool has_geom = false;
    int32_t n_subjects = 0, M = 0;
    int64_t N = 0, P = 0;
    std::vector<int64_t> gauss_off;
    std::vector<int32_t> slice_subject, H, W;
    std::vector<float> spacing, fwhm, rot0, trans0;
    std::vector<int64_t> pix_off;
    int32_t max_subject_slices = 0;

    svr_config cfg{16, 128, 0, 3.0f, 1};

    // tile tables (host)
    int32_t n_tiles = 0, key_bits = 1;
    int32_t n_blocks = 0;

    // device tables
    DevBuf<SliceGeo> d_geo;
    DevBuf<SlicePose> d_pose;
    DevBuf<SlicePlane> d_plane;
    DevBuf<SubjectInfo> d_subj;
    DevBuf<GaussBlock> d_blocks;
    DevBuf<int32_t> d_tile_slice;
    DevBuf<int4> d_tile_org;       // per tile origin, see TileOrg
    DevBuf<int2> d_counts, d_offsets;
    DevBuf<char> d_scan_tmp;
    DevBuf<long long> d_totals;
    long long* h_totals = nullptr;
    DevBuf<Record> d_rec;
    DevBuf<int2> d_rec_inst;
    DevBuf<float4> d_inst_grad;
    DevBuf<uint32_t> d_keys, d_vals, d_keys2, d_vals2, d_idx, d_idx2;
    DevBuf<char> d_sort_tmp;
    DevBuf<int2> d_ranges;
    DevBuf<float> d_tile_sse, d_partial, d_msum, d_slice_sse, d_pose_acc;
    DevBuf<int> d_work, d_fallback;
    int32_t loss_kind = 0;        // SVR_LOSS_MSE / SVR_LOSS_L1
    DevBuf<float> d_regpart;      // scale-regulariser block partials
    DevBuf<float> d_bias_scratch; // bias-field adjoint partials
    DevBuf<float> d_pose_part, d_pose_pp;  // projection adjoint: pose sums per workgroup, per 256 workgroups
    DevBuf<int4> d_pose_w1;                // their first-level work items (subject, columns, parts)
    DevBuf<int2> d_pose_w2;                // second-level work items (subject, columns)
    int64_t pose_part_floats = 0, pose_pp_floats = 0;
    int32_t n_pose_w1 = 0, n_pose_w2 = 0;
    DevBuf<int32_t> d_dens_n, d_dens_pos;   // densification: outputs per Gaussian and their scan
    DevBuf<int64_t> d_dens_off;             // densification: new per-subject offsets
    DevBuf<long long> d_dens_tot;
    DevBuf<float> d_fwd_part;     // chunked record-per-lane forward: two tile partials per instance chunk
    DevBuf<uint32_t> d_smask;  // plane-test survivor bits per Gaussian
    // content-adaptive initialisation (allocated on first use)
    DevBuf<InitSlice> d_init_tab;
    DevBuf<SlicePose> d_init_pose;
    DevBuf<int64_t> d_init_subpix, d_init_cdf, d_init_bsum, d_init_base, d_init_total;
    DevBuf<double> d_init_g;
    DevBuf<unsigned long long> d_init_gmax;
    // normalised Top-K model (allocated on first use)
    DevBuf<TopkGauss> d_topk_gauss;
    DevBuf<TopkSlice> d_topk_slices;
    DevBuf<SlicePose> d_topk_pose;
    DevBuf<uint32_t> d_topk_bb;
    DevBuf<TopkGrid> d_topk_grid;
    DevBuf<int2> d_topk_cells, d_topk_granges;
    DevBuf<float4> d_topk_smean;
    DevBuf<uint32_t> d_topk_ck, d_topk_cv, d_topk_ck2, d_topk_cv2;
    DevBuf<uint32_t> d_topk_pk, d_topk_pv, d_topk_pk2, d_topk_pv2;
    DevBuf<char> d_topk_sort_tmp;
    DevBuf<float2> d_topk_state;
    DevBuf<float> d_topk_partial, d_topk_pose_acc, d_topk_msum;
    DevBuf<int> d_topk_status;
    DevBuf<int> d_topk_flag, d_topk_aoff;
    DevBuf<uint8_t> d_topk_active;
    DevBuf<int32_t> d_topk_act, d_topk_act_off;
    DevBuf<char> d_topk_scan_tmp;
    DevBuf<long long> d_topk_tot;
    int64_t topk_n_act = 0;
    int32_t topk_max_act = 1;
    DevBuf<int32_t> d_topk_iperm, d_topk_lint;
    DevBuf<int64_t> d_topk_qoff;
    DevBuf<float4> d_topk_pxw;
    DevBuf<float2> d_topk_pyd;
    const uint32_t* topk_perm = nullptr;
    DevBuf<float> d_sl_scratch, d_sl_msum;   // per-slice outlier terms
    const uint32_t* topk_gpix = nullptr;
    const int32_t* topk_nbr = nullptr;
    int32_t topk_K = 0;
    bool topk_built = false, topk_forwarded = false;
    int64_t topk_split_tiles = 0;
    DevBuf<unsigned long long> d_incut;
    DevBuf<uint32_t> d_tkeys, d_tvals, d_tkeys2, d_tvals2;
    DevBuf<char> d_tsort_tmp;
    const int32_t* tile_order = nullptr;

    // fixed-capacity binning (cap_rec > 0): no count read-back in project_bin
    int64_t cap_rec = 0, cap_inst = 0;
    int check_flags = 0;            // SVR_CHECK_*
    DevBuf<DevStatus> d_status;     // conditions recorded on the device
    DevStatus* h_status = nullptr;  // pinned read-back of d_status

    // binning state
    bool binned = false;
    int64_t n_rec = 0, n_inst = 0, n_cand = 0;
    const uint32_t* sorted_vals = nullptr;
    const uint32_t* sorted_idx = nullptr;
    const uint32_t* sorted_keys = nullptr;
    svr_params params{};
    bool count_pairs = false;
    bool incut_pending = false;
    int64_t n_incut = -1;

    std::map<std::string, svr_config> tune_cache;

    // stage timing
    bool timing = false;
    uint32_t timing_mask = 0xffffffffu;  // bit s: stage s is bracketed by events while timing
    std::vector<hipEvent_t> ev_free;
    struct Pending { int stage; hipEvent_t a, b; };
    std::vector<Pending> pending;
    int64_t t_calls[ST_COUNT] = {0};
    double t_ms[ST_COUNT] = {0.0};
};

namespace {

int fail(svr_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return fail((ctx), SVR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    } while (0)

template <class T>
hipError_t ensure(DevBuf<T>& b, size_t need, bool exact = false) {
    if (need == 0) need = 1;
    if (b.cap >= need) return hipSuccess;
    size_t n = exact ? need : std::max(need, b.cap + b.cap / 2);
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc((void**)&b.p, n * sizeof(T));
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.cap = n;
    return hipSuccess;
}

template <class T>
void release(DevBuf<T>& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

int enter(svr_ctx* c) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (c->host_only) return fail(c, SVR_ERR_NODEVICE, "host-only context has no GPU");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, SVR_ERR_HIP, "hipSetDevice(%d): %s", c->device, hipGetErrorString(e));
    return SVR_OK;
}

bool valid_config(const svr_config& g) {
    return (g.tile == 8 || g.tile == 16 || g.tile == 32) && g.batch >= 32 && g.batch <= 256 &&
           (g.batch % 32) == 0 && (g.persistent == 0 || g.persistent == 1) && g.cutoff > 0.f &&
           g.cutoff <= 8.f && isfinite(g.cutoff) && (g.forward_mode >= 0 && g.forward_mode <= 2);
}

// Builds host tile tables and (if a device is present) uploads every table.
int build_tables(svr_ctx* c) {
    const int T = c->cfg.tile;
    std::vector<SliceGeo> geo(c->M);
    int64_t tiles = 0;
    for (int i = 0; i < c->M; ++i) {
        SliceGeo& g = geo[i];
        for (int k = 0; k < 9; ++k) g.R0[k] = c->rot0[9 * i + k];
        for (int k = 0; k < 3; ++k) g.t0[k] = c->trans0[3 * i + k];
        for (int k = 0; k < 3; ++k) {
            const float sg = c->fwhm[3 * i + k] / 2.355f;
            g.sig2[k] = sg * sg;
        }
        g.dx = c->spacing[2 * i];
        g.dy = c->spacing[2 * i + 1];
        g.H = c->H[i];
        g.W = c->W[i];
        g.ntx = (g.W + T - 1) / T;
        g.nty = (g.H + T - 1) / T;
        g.tile_base = (int32_t)tiles;
        g.subject = c->slice_subject[i];
        g.pix_off = c->pix_off[i];
        tiles += (int64_t)g.ntx * g.nty;
    }
    if (tiles > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "tile count %lld exceeds 2^31-1", (long long)tiles);
    c->n_tiles = (int32_t)tiles;
    // tile part: 2^bits > n_tiles, so the all-ones padding key sorts after
    // every tile; plus the size-class bits below it
    int kb = 1;
    while (kb < 32 && (1LL << kb) <= tiles) ++kb;
    if (kb + kClassBits > 32) return fail(c, SVR_ERR_CAPACITY, "tile count %lld too large for the sort key", (long long)tiles);
    c->key_bits = kb + kClassBits;
    std::vector<int32_t> tile_slice((size_t)tiles);
    // per tile: global pixel id of its origin (two ints), x0 | y0 << 16 and
    // slice width | valid width << 16 | valid height << 24 (see TileOrg)
    std::vector<int4> tile_org((size_t)tiles);
    for (int i = 0; i < c->M; ++i) {
        if (geo[i].W > 0xffff || geo[i].H > 0xffff)
            return fail(c, SVR_ERR_CAPACITY, "slice %d is %d x %d pixels; at most 65535 per side", i, geo[i].H,
                        geo[i].W);
        for (int t = 0; t < geo[i].ntx * geo[i].nty; ++t) {
            tile_slice[geo[i].tile_base + t] = i;
            const int ty = t / geo[i].ntx, tx = t - ty * geo[i].ntx;
            const int x0 = tx * T, y0 = ty * T;
            const int64_t base = geo[i].pix_off + (int64_t)y0 * geo[i].W + x0;
            const int vw = std::min(T, geo[i].W - x0), vh = std::min(T, geo[i].H - y0);
            tile_org[geo[i].tile_base + t] = make_int4((int)(uint32_t)(uint64_t)base, (int)((uint64_t)base >> 32),
                                                       x0 | (y0 << 16), geo[i].W | (vw << 16) | (vh << 24));
        }
    }
    std::vector<SubjectInfo> subj(c->n_subjects);
    std::vector<GaussBlock> blocks;
    for (int s = 0; s < c->n_subjects; ++s) {
        subj[s] = SubjectInfo{};
        subj[s].g_begin = c->gauss_off[s];
        subj[s].g_end = c->gauss_off[s + 1];
        subj[s].part0 = kProjParts * (int32_t)blocks.size();
        for (int64_t g0 = subj[s].g_begin; g0 < subj[s].g_end; g0 += kGaussBlock) {
            GaussBlock b;
            b.g_begin = g0;
            b.g_end = std::min(g0 + kGaussBlock, subj[s].g_end);
            b.subject = s;
            b.pad = 0;
            blocks.push_back(b);
        }
    }
    {
        int i = 0;
        for (int s = 0; s < c->n_subjects; ++s) {
            subj[s].s_begin = i;
            while (i < c->M && c->slice_subject[i] == s) ++i;
            subj[s].s_end = i;
        }
    }
    c->n_blocks = (int32_t)blocks.size();
    // the projection adjoint's two-level pose reduction: rows of 6 ns sums
    // per workgroup, then per 256 workgroups (work items of 64 columns)
    std::vector<int4> w1;
    std::vector<int2> w2;
    int64_t pose_rows = 0, pp_rows = 0;
    for (int s = 0; s < c->n_subjects; ++s) {
        const int32_t nb_s = (int32_t)((subj[s].g_end - subj[s].g_begin + kGaussBlock - 1) / kGaussBlock);
        const int64_t C = 6 * (int64_t)(subj[s].s_end - subj[s].s_begin);
        subj[s].nparts = kProjParts * nb_s;
        subj[s].nrc = (subj[s].nparts + kPoseRowChunk - 1) / kPoseRowChunk;
        subj[s].pose_base = pose_rows;
        subj[s].pp_base = pp_rows;
        pose_rows += (int64_t)subj[s].nparts * C;
        pp_rows += (int64_t)subj[s].nrc * C;
        for (int cg = 0; cg < (int)((C + 63) / 64); ++cg) {
            for (int rc = 0; rc < subj[s].nrc; ++rc) w1.push_back(make_int4(s, cg, rc, 0));
            w2.push_back(make_int2(s, cg));
        }
    }
    c->pose_part_floats = pose_rows;
    c->pose_pp_floats = pp_rows;
    c->n_pose_w1 = (int32_t)w1.size();
    c->n_pose_w2 = (int32_t)w2.size();
    if (c->host_only) return SVR_OK;
    hipStream_t st = c->stream;
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, ensure(c->d_geo, geo.size()));
    HIPCHK(c, ensure(c->d_pose, geo.size()));
    HIPCHK(c, ensure(c->d_plane, geo.size()));
    HIPCHK(c, ensure(c->d_subj, subj.size()));
    HIPCHK(c, ensure(c->d_blocks, blocks.size()));
    HIPCHK(c, ensure(c->d_tile_slice, tile_slice.size()));
    HIPCHK(c, ensure(c->d_tile_org, tile_org.size()));
    HIPCHK(c, ensure(c->d_ranges, tile_slice.size()));
    HIPCHK(c, ensure(c->d_tile_sse, tile_slice.size()));
    HIPCHK(c, ensure(c->d_slice_sse, (size_t)c->M));
    HIPCHK(c, ensure(c->d_pose_acc, (size_t)c->M * 6));
    HIPCHK(c, ensure(c->d_pose_w1, std::max<size_t>(w1.size(), 1)));
    HIPCHK(c, ensure(c->d_pose_w2, std::max<size_t>(w2.size(), 1)));
    if (!w1.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_pose_w1.p, w1.data(), w1.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    if (!w2.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_pose_w2.p, w2.data(), w2.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIPCHK(c, ensure(c->d_counts, (size_t)c->N));
    HIPCHK(c, ensure(c->d_offsets, (size_t)c->N));
    if (!geo.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_geo.p, geo.data(), geo.size() * sizeof(SliceGeo), hipMemcpyHostToDevice, st));
    if (!subj.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_subj.p, subj.data(), subj.size() * sizeof(SubjectInfo), hipMemcpyHostToDevice, st));
    if (!blocks.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_blocks.p, blocks.data(), blocks.size() * sizeof(GaussBlock), hipMemcpyHostToDevice, st));
    if (!tile_slice.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_tile_slice.p, tile_slice.data(), tile_slice.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!tile_org.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_tile_org.p, tile_org.data(), tile_org.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->binned = false;
    return SVR_OK;
}

hipEvent_t take_event(svr_ctx* c) {
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one stage with events on the context stream when timing is on.
struct StageScope {
    svr_ctx* c;
    int stage;
    hipEvent_t a = nullptr;
    StageScope(svr_ctx* ctx, int s) : c(ctx), stage(s) {
        if (c->timing && ((c->timing_mask >> s) & 1u)) {
            a = take_event(c);
            if (a && hipEventRecord(a, c->stream) != hipSuccess) a = nullptr;
        }
    }
    ~StageScope() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (b && hipEventRecord(b, c->stream) == hipSuccess) c->pending.push_back({stage, a, b});
        else c->ev_free.push_back(a);
    }
};

int fold_timing(svr_ctx* c) {
    if (c->pending.empty()) return SVR_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->t_ms[p.stage] += ms;
            c->t_calls[p.stage] += 1;
        }
        c->ev_free.push_back(p.a);
        c->ev_free.push_back(p.b);
    }
    c->pending.clear();
    return SVR_OK;
}

ProjectArgs project_args(svr_ctx* c) {
    ProjectArgs a;
    a.mean = c->params.mean;
    a.log_scale = c->params.log_scale;
    a.quat = c->params.quat;
    a.amp = c->params.amp;
    a.geo = c->d_geo.p;
    a.pose = c->d_pose.p;
    a.plane = c->d_plane.p;
    a.subj = c->d_subj.p;
    a.blocks = c->d_blocks.p;
    a.n_blocks = c->n_blocks;
    a.tile = c->cfg.tile;
    a.tau = c->cfg.cutoff;
    a.smask = c->d_smask.p;
    a.smask_words = std::max((c->max_subject_slices + 31) / 32, 1);
    return a;
}

RenderArgs render_args(svr_ctx* c) {
    RenderArgs a;
    a.geo = c->d_geo.p;
    a.tile_slice = c->d_tile_slice.p;
    a.tile_org = c->d_tile_org.p;
    a.ranges = c->d_ranges.p;
    a.inst_rec = c->sorted_vals;
    a.inst_idx = c->sorted_idx;
    a.inst_key = c->sorted_keys;
    a.n_inst = c->n_inst;
    a.rec = c->d_rec.p;
    a.tile_order = c->cfg.persistent ? c->tile_order : nullptr;
    a.n_tiles = c->n_tiles;
    a.tile = c->cfg.tile;
    a.batch = c->cfg.batch;
    a.persistent = c->cfg.persistent;
    a.forward_mode = c->cfg.forward_mode;
    a.loss_kind = c->loss_kind;
    a.tau2 = c->cfg.cutoff * c->cfg.cutoff;
    a.etau = expf(-0.5f * a.tau2);
    a.n_cu = c->n_cu;
    return a;
}

// Persistent-mode work order: tiles by decreasing instance count.
int build_tile_order(svr_ctx* c) {
    hipStream_t st = c->stream;
    const size_t nt = (size_t)c->n_tiles;
    HIPCHK(c, ensure(c->d_tkeys, nt));
    HIPCHK(c, ensure(c->d_tvals, nt));
    HIPCHK(c, ensure(c->d_tkeys2, nt));
    HIPCHK(c, ensure(c->d_tvals2, nt));
    HIPCHK(c, ensure(c->d_tsort_tmp, sort_tmp_bytes((int64_t)nt)));
    bool alt = false;
    {
        StageScope sc(c, ST_TILE_ORDER);
        HIPCHK(c, launch_tile_cost_keys(c->d_ranges.p, c->n_tiles, c->d_tkeys.p, c->d_tvals.p, st));
        HIPCHK(c, launch_radix_sort(c->d_tkeys.p, c->d_tvals.p, c->d_tkeys2.p, c->d_tvals2.p, (int64_t)nt, 16,
                                    c->d_tsort_tmp.p, &alt, st));
    }
    c->tile_order = (const int32_t*)(alt ? c->d_tvals2.p : c->d_tvals.p);
    return SVR_OK;
}

// Binning buffers for nrec records and ninst instance slots.
int ensure_bin_buffers(svr_ctx* c, int64_t nrec, int64_t ninst) {
    HIPCHK(c, ensure(c->d_fallback, (size_t)std::max(c->n_blocks, 1)));
    HIPCHK(c, ensure(c->d_rec, (size_t)nrec));
    HIPCHK(c, ensure(c->d_rec_inst, (size_t)nrec));
    HIPCHK(c, ensure(c->d_inst_grad, 2 * (size_t)ninst));
    HIPCHK(c, ensure(c->d_keys, (size_t)ninst));
    HIPCHK(c, ensure(c->d_vals, (size_t)ninst));
    HIPCHK(c, ensure(c->d_keys2, (size_t)ninst));
    HIPCHK(c, ensure(c->d_vals2, (size_t)ninst));
    HIPCHK(c, ensure(c->d_idx, (size_t)ninst));
    HIPCHK(c, ensure(c->d_idx2, (size_t)ninst));
    HIPCHK(c, ensure(c->d_sort_tmp, sort_tmp_bytes(ninst)));
    return SVR_OK;
}

// Finite check of the Gaussian parameters and poses (SVR_CHECK_FINITE).
int check_params_finite(svr_ctx* c, const svr_params* p) {
    hipStream_t st = c->stream;
    HIPCHK(c, launch_check_finite(p->mean, 3 * c->N, c->d_status.p, st));
    HIPCHK(c, launch_check_finite(p->log_scale, 3 * c->N, c->d_status.p, st));
    HIPCHK(c, launch_check_finite(p->quat, 4 * c->N, c->d_status.p, st));
    HIPCHK(c, launch_check_finite(p->amp, c->N, c->d_status.p, st));
    HIPCHK(c, launch_check_finite(p->pose, 6 * (int64_t)c->M, c->d_status.p, st));
    return SVR_OK;
}

int project_bin_impl(svr_ctx* c, const svr_params* p) {
    hipStream_t st = c->stream;
    const bool fixed = c->cap_rec > 0;
    c->params = *p;
    c->binned = false;
    c->incut_pending = false;
    c->n_incut = -1;
    if (c->check_flags & SVR_CHECK_FINITE) {
        int rc = check_params_finite(c, p);
        if (rc != SVR_OK) return rc;
    }
    {
        StageScope sc(c, ST_SLICE_POSE);
        HIPCHK(c, launch_slice_pose(c->d_geo.p, p->pose, c->d_pose.p, c->M, st, c->d_plane.p));
    }
    HIPCHK(c, ensure(c->d_smask, (size_t)std::max<int64_t>(c->N, 1) * (size_t)std::max((c->max_subject_slices + 31) / 32, 1)));
    ProjectArgs pa = project_args(c);
    {
        StageScope sc(c, ST_CULL_COUNT);
        HIPCHK(c, launch_cull_count(pa, c->d_counts.p, st));
    }
    HIPCHK(c, ensure(c->d_scan_tmp, scan_tmp_bytes(c->N) + 64));
    HIPCHK(c, ensure(c->d_totals, 2));
    {
        StageScope sc(c, ST_SCAN);
        HIPCHK(c, launch_scan_int2(c->d_counts.p, c->d_offsets.p, c->N, c->d_totals.p, c->d_scan_tmp.p, st));
    }
    int64_t nrec, ninst;
    if (fixed) {
        // counts stay on the device; an iteration that needs more than the
        // capacity bins nothing and records the needed counts
        HIPCHK(c, launch_fixed_capacity(c->d_totals.p, c->cap_rec, c->cap_inst, c->d_counts.p, c->d_offsets.p, c->N,
                                         c->d_status.p, st));
        nrec = c->cap_rec;
        ninst = c->cap_inst;
    } else {
        HIPCHK(c, hipMemcpyAsync(c->h_totals, c->d_totals.p, 2 * sizeof(long long), hipMemcpyDeviceToHost, st));
        if (c->check_flags & SVR_CHECK_FINITE)
            HIPCHK(c, hipMemcpyAsync(c->h_status, c->d_status.p, sizeof(DevStatus), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if ((c->check_flags & SVR_CHECK_FINITE) && (c->h_status->bits & kStatusNonfinite)) {
            HIPCHK(c, launch_fill_zero(c->d_status.p, sizeof(DevStatus), st));
            return fail(c, SVR_ERR_NONFINITE, "a Gaussian parameter or slice pose is NaN or infinite");
        }
        nrec = c->h_totals[0];
        ninst = c->h_totals[1];
        if (nrec > 0x7fffffffLL || ninst > 0x7fffffffLL)
            return fail(c, SVR_ERR_CAPACITY, "records (%lld) or instances (%lld) exceed 2^31-1", (long long)nrec,
                        (long long)ninst);
    }
    c->n_rec = nrec;
    c->n_inst = ninst;
    int64_t cand = 0;
    for (int s = 0; s < c->n_subjects; ++s) {
        int ns = 0;
        for (int i = 0; i < c->M; ++i) ns += (c->slice_subject[i] == s);
        cand += (c->gauss_off[s + 1] - c->gauss_off[s]) * (int64_t)ns;
    }
    c->n_cand = cand;
    {
        int rc = ensure_bin_buffers(c, nrec, ninst);
        if (rc != SVR_OK) return rc;
    }
    {
        StageScope sc(c, ST_EMIT);
        HIPCHK(c, launch_emit(pa, c->d_counts.p, c->d_offsets.p, c->d_rec.p, c->d_rec_inst.p, c->d_keys.p,
                              c->d_vals.p, c->d_fallback.p, fixed ? &c->d_status.p->overflow : nullptr, st));
        if (fixed)
            HIPCHK(c, launch_pad_instances(c->d_keys.p, c->d_vals.p, ninst, c->d_totals.p, c->d_status.p, st));
    }
    bool alt = false;
    {
        StageScope sc(c, ST_SORT);
        // tile bits only: the shape class (low bits) is ordered per tile by the tile kernels
        HIPCHK(c, launch_radix_sort(c->d_keys.p, c->d_vals.p, c->d_keys2.p, c->d_vals2.p, ninst, c->key_bits,
                                    c->d_sort_tmp.p, &alt, st, c->d_idx.p, c->d_idx2.p, kClassBits));
    }
    const uint32_t* sk = alt ? c->d_keys2.p : c->d_keys.p;
    // each tile's instances then go in shape-class order into the other buffers
    uint32_t* ko = alt ? c->d_keys.p : c->d_keys2.p;
    uint32_t* vo = alt ? c->d_vals.p : c->d_vals2.p;
    uint32_t* xo = alt ? c->d_idx.p : c->d_idx2.p;
    {
        StageScope sc(c, ST_TILE_RANGES);
        HIPCHK(c, launch_tile_ranges(sk, ninst, c->d_ranges.p, c->n_tiles, ko, st));
    }
    {
        StageScope sc(c, ST_CLASS_ORDER);
        HIPCHK(c, launch_class_order(sk, alt ? c->d_vals2.p : c->d_vals.p, alt ? c->d_idx2.p : c->d_idx.p,
                                     c->d_ranges.p, c->n_tiles, ko, vo, xo, st));
        c->sorted_keys = ko;
        c->sorted_vals = vo;
        c->sorted_idx = xo;
    }
    if (c->cfg.persistent) {
        int rc = build_tile_order(c);
        if (rc != SVR_OK) return rc;
    }
    c->binned = true;
    return SVR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free sort (svr_sort_pairs_noalloc).  Its scratch -- ping-pong
// keys and values and the pass histograms for up to SVR_SORT_NOALLOC_MAX
// pairs -- is the file-scope device array below, which every GPU the library
// runs on holds until the process ends.  In host code the array's name is a
// host-side stand-in, not a device address: kernels and copies get the
// address hipGetSymbolAddress returns on each device, looked up once per
// device when the first context on it is created (noalloc_setup).
namespace {
constexpr int64_t kNoallocMax = SVR_SORT_NOALLOC_MAX;
constexpr size_t kNoallocKV = (size_t)kNoallocMax * sizeof(uint32_t);  // keys or values
constexpr size_t kNoallocTmp = (size_t)3 << 20;                        // pass histograms and scan partials
constexpr size_t kNoallocBytes = 2 * kNoallocKV + kNoallocTmp;
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocDevices] = {};
hipError_t g_noalloc_err[kNoallocDevices] = {};
bool g_noalloc_done[kNoallocDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// Looks up this device's copy of the scratch array; `device` must be current.
static void noalloc_setup(int device) {
    if (device < 0 || device >= kNoallocDevices) return;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_done[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    g_noalloc_err[device] = e;
    g_noalloc_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_noalloc_done[device] = true;
}

// ---------------------------------------------------------------------------
extern "C" {

int svr_abi_version(void) { return SVR_ABI_VERSION; }

const char* svr_status_string(int s) {
    switch (s) {
        case SVR_OK: return "SVR_OK";
        case SVR_ERR_ARG: return "SVR_ERR_ARG";
        case SVR_ERR_HIP: return "SVR_ERR_HIP";
        case SVR_ERR_CAPACITY: return "SVR_ERR_CAPACITY";
        case SVR_ERR_STATE: return "SVR_ERR_STATE";
        case SVR_ERR_NODEVICE: return "SVR_ERR_NODEVICE";
        case SVR_ERR_NONFINITE: return "SVR_ERR_NONFINITE";
        default: return "SVR_ERR_UNKNOWN";
    }
}

int svr_ctx_create(svr_ctx** out, int device, void* hip_stream) {
    if (!out) return SVR_ERR_ARG;
    *out = nullptr;
    if (device < -1) return SVR_ERR_ARG;
    svr_ctx* c = new (std::nothrow) svr_ctx();
    if (!c) return SVR_ERR_CAPACITY;
    if (device == -1) {
        c->host_only = true;
        *out = c;
        return SVR_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
        delete c;
        return SVR_ERR_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SVR_ERR_HIP;
    }
    c->device = device;
    c->host_only = false;
    c->stream = (hipStream_t)hip_stream;
    noalloc_setup(device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->n_cu = cus;
    if (hipHostMalloc((void**)&c->h_totals, 4 * sizeof(long long), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SVR_ERR_HIP;
    }
    if (hipHostMalloc((void**)&c->h_status, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess ||
        ensure(c->d_status, 1) != hipSuccess ||
        launch_fill_zero(c->d_status.p, sizeof(DevStatus), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        if (c->h_status) (void)hipHostFree(c->h_status);
        release(c->d_status);
        (void)hipHostFree(c->h_totals);
        delete c;
        return SVR_ERR_HIP;
    }
    *out = c;
    return SVR_OK;
}

int svr_ctx_destroy(svr_ctx* c) {
    if (!c) return SVR_OK;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        release(c->d_geo); release(c->d_pose); release(c->d_plane); release(c->d_subj); release(c->d_blocks);
        release(c->d_tile_slice); release(c->d_tile_org); release(c->d_counts); release(c->d_offsets); release(c->d_scan_tmp);
        release(c->d_totals); release(c->d_rec); release(c->d_rec_inst); release(c->d_inst_grad);
        release(c->d_idx); release(c->d_idx2); release(c->d_keys);
        release(c->d_vals); release(c->d_keys2); release(c->d_vals2); release(c->d_sort_tmp);
        release(c->d_ranges); release(c->d_tile_sse); release(c->d_partial); release(c->d_msum);
        release(c->d_slice_sse); release(c->d_pose_acc); release(c->d_work); release(c->d_incut);
        release(c->d_fallback);
        release(c->d_tkeys); release(c->d_tvals); release(c->d_tkeys2); release(c->d_tvals2);
        release(c->d_tsort_tmp);
        release(c->d_dens_n); release(c->d_dens_pos); release(c->d_dens_off); release(c->d_dens_tot);
        release(c->d_pose_part); release(c->d_pose_pp); release(c->d_pose_w1); release(c->d_pose_w2);
        release(c->d_regpart); release(c->d_bias_scratch); release(c->d_smask); release(c->d_fwd_part);
        release(c->d_init_tab); release(c->d_init_pose); release(c->d_init_subpix); release(c->d_init_cdf);
        release(c->d_init_bsum); release(c->d_init_base); release(c->d_init_total); release(c->d_init_g);
        release(c->d_init_gmax);
        release(c->d_topk_gauss); release(c->d_topk_slices); release(c->d_topk_pose); release(c->d_topk_bb);
        release(c->d_topk_grid); release(c->d_topk_cells); release(c->d_topk_granges); release(c->d_topk_smean);
        release(c->d_topk_ck); release(c->d_topk_cv); release(c->d_topk_ck2); release(c->d_topk_cv2);
        release(c->d_topk_pk); release(c->d_topk_pv); release(c->d_topk_pk2); release(c->d_topk_pv2);
        release(c->d_topk_sort_tmp); release(c->d_topk_state); release(c->d_topk_partial);
        release(c->d_topk_pose_acc); release(c->d_topk_msum); release(c->d_topk_status);
        release(c->d_sl_scratch); release(c->d_sl_msum);
        release(c->d_topk_flag); release(c->d_topk_aoff); release(c->d_topk_active); release(c->d_topk_act);
        release(c->d_topk_act_off); release(c->d_topk_scan_tmp); release(c->d_topk_tot);
        release(c->d_topk_iperm); release(c->d_topk_lint); release(c->d_topk_qoff); release(c->d_topk_pxw);
        release(c->d_topk_pyd);
        if (c->h_totals) (void)hipHostFree(c->h_totals);
        if (c->h_status) (void)hipHostFree(c->h_status);
        release(c->d_status);
        for (auto& p : c->pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (auto e : c->ev_free) (void)hipEventDestroy(e);
    }
    delete c;
    return SVR_OK;
}

int svr_set_stream(svr_ctx* c, void* s) {
    if (!c) return SVR_ERR_ARG;
    c->stream = (hipStream_t)s;
    return SVR_OK;
}

const char* svr_last_error(const svr_ctx* c) { return c ? c->err.c_str() : "null context"; }

int svr_set_geometry(svr_ctx* c, const svr_geometry* g) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!g) return fail(c, SVR_ERR_ARG, "geometry is NULL");
    if (g->n_subjects < 1) return fail(c, SVR_ERR_ARG, "n_subjects must be >= 1");
    if (g->n_slices < 0) return fail(c, SVR_ERR_ARG, "n_slices must be >= 0");
    if (!g->gauss_offsets) return fail(c, SVR_ERR_ARG, "gauss_offsets is NULL");
    if (g->n_slices > 0 && (!g->slice_subject || !g->height || !g->width || !g->spacing || !g->psf_fwhm ||
                            !g->rot0 || !g->trans0))
        return fail(c, SVR_ERR_ARG, "a per-slice array is NULL");
    if (g->gauss_offsets[0] != 0) return fail(c, SVR_ERR_ARG, "gauss_offsets[0] must be 0");
    for (int s = 0; s < g->n_subjects; ++s)
        if (g->gauss_offsets[s + 1] < g->gauss_offsets[s])
            return fail(c, SVR_ERR_ARG, "gauss_offsets must be nondecreasing (subject %d)", s);
    const int M = g->n_slices;
    int64_t P = 0;
    std::vector<int> per_subject(g->n_subjects, 0);
    for (int i = 0; i < M; ++i) {
        if (g->slice_subject[i] < 0 || g->slice_subject[i] >= g->n_subjects)
            return fail(c, SVR_ERR_ARG, "slice %d: subject %d out of range", i, g->slice_subject[i]);
        if (i > 0 && g->slice_subject[i] < g->slice_subject[i - 1])
            return fail(c, SVR_ERR_ARG, "slices must be grouped by nondecreasing subject (slice %d)", i);
        if (g->height[i] < 1 || g->width[i] < 1)
            return fail(c, SVR_ERR_ARG, "slice %d: size %dx%d must be positive", i, g->height[i], g->width[i]);
        if (!(g->spacing[2 * i] > 0.f) || !(g->spacing[2 * i + 1] > 0.f) || !isfinite(g->spacing[2 * i]) ||
            !isfinite(g->spacing[2 * i + 1]))
            return fail(c, SVR_ERR_ARG, "slice %d: spacing must be positive and finite", i);
        for (int k = 0; k < 3; ++k)
            if (!(g->psf_fwhm[3 * i + k] >= 0.f) || !isfinite(g->psf_fwhm[3 * i + k]))
                return fail(c, SVR_ERR_ARG, "slice %d: PSF FWHM must be >= 0 and finite", i);
        for (int k = 0; k < 9; ++k)
            if (!isfinite(g->rot0[9 * i + k])) return fail(c, SVR_ERR_ARG, "slice %d: rot0 not finite", i);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(g->trans0[3 * i + k])) return fail(c, SVR_ERR_ARG, "slice %d: trans0 not finite", i);
        P += (int64_t)g->height[i] * g->width[i];
        per_subject[g->slice_subject[i]]++;
    }
    if (P > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "pixel count %lld exceeds 2^31-1", (long long)P);
    int maxs = 0;
    for (int s = 0; s < g->n_subjects; ++s) maxs = std::max(maxs, per_subject[s]);
    if (maxs > kMaxSubjectSlices)
        return fail(c, SVR_ERR_CAPACITY, "a subject has %d slices (limit %d)", maxs, kMaxSubjectSlices);
    c->n_subjects = g->n_subjects;
    c->M = M;
    c->N = g->gauss_offsets[g->n_subjects];
    c->P = P;
    c->gauss_off.assign(g->gauss_offsets, g->gauss_offsets + g->n_subjects + 1);
    c->slice_subject.assign(g->slice_subject, g->slice_subject + M);
    c->H.assign(g->height, g->height + M);
    c->W.assign(g->width, g->width + M);
    c->spacing.assign(g->spacing, g->spacing + 2 * M);
    c->fwhm.assign(g->psf_fwhm, g->psf_fwhm + 3 * M);
    c->rot0.assign(g->rot0, g->rot0 + 9 * M);
    c->trans0.assign(g->trans0, g->trans0 + 3 * M);
    c->pix_off.assign(M + 1, 0);
    for (int i = 0; i < M; ++i) c->pix_off[i + 1] = c->pix_off[i] + (int64_t)g->height[i] * g->width[i];
    c->max_subject_slices = maxs;
    c->has_geom = true;
    c->binned = false;
    c->topk_built = false;
    c->topk_forwarded = false;
    if (!c->host_only && hipSetDevice(c->device) != hipSuccess)
        return fail(c, SVR_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    return build_tables(c);
}

int64_t svr_num_pixels(const svr_ctx* c) { return (c && c->has_geom) ? c->P : 0; }

int svr_set_config(svr_ctx* c, const svr_config* cfg) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!cfg) return fail(c, SVR_ERR_ARG, "config is NULL");
    if (!valid_config(*cfg))
        return fail(c, SVR_ERR_ARG, "invalid config (tile %d, batch %d, persistent %d, cutoff %g, forward_mode %d)",
                    cfg->tile, cfg->batch, cfg->persistent, (double)cfg->cutoff, cfg->forward_mode);
    const bool retile = cfg->tile != c->cfg.tile;
    const bool recut = cfg->cutoff != c->cfg.cutoff;
    const bool repersist = cfg->persistent != c->cfg.persistent;
    c->cfg = *cfg;
    if (retile || recut) c->binned = false;
    if (retile && c->has_geom) {
        if (!c->host_only) (void)hipSetDevice(c->device);
        int rc = build_tables(c);
        if (rc != SVR_OK) return rc;
    }
    if (repersist && c->binned && c->cfg.persistent && !c->host_only) {
        (void)hipSetDevice(c->device);
        int rc = build_tile_order(c);
        if (rc != SVR_OK) return rc;
    }
    return SVR_OK;
}

int svr_get_config(const svr_ctx* c, svr_config* cfg) {
    if (!c || !cfg) return SVR_ERR_ARG;
    *cfg = c->cfg;
    return SVR_OK;
}

int svr_project_bin(svr_ctx* c, const svr_params* p) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!p) return fail(c, SVR_ERR_ARG, "params is NULL");
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "svr_set_geometry has not been called");
    if (c->N > 0 && (!p->mean || !p->log_scale || !p->quat || !p->amp))
        return fail(c, SVR_ERR_ARG, "a Gaussian parameter pointer is NULL");
    if (c->M > 0 && !p->pose) return fail(c, SVR_ERR_ARG, "pose is NULL");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    return project_bin_impl(c, p);
}

int svr_forward(svr_ctx* c, const float* target, const float* mask, float* pred, float* loss,
                float* slice_sse, float* grad_pred) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!pred) return fail(c, SVR_ERR_ARG, "pred is NULL");
    const bool want_loss = loss || slice_sse || grad_pred;
    if (want_loss && (!target || !mask))
        return fail(c, SVR_ERR_ARG, "loss outputs requested without target and mask");
    if (!c->binned) return fail(c, SVR_ERR_STATE, "svr_project_bin has not been called");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    hipStream_t st = c->stream;
    RenderArgs ra = render_args(c);
    HIPCHK(c, ensure(c->d_msum, 4));
    HIPCHK(c, ensure(c->d_partial, 1024));
    HIPCHK(c, ensure(c->d_work, 4));
    HIPCHK(c, ensure(c->d_incut, 1));
    const size_t npart = forward_partial_floats(ra);
    if (npart) HIPCHK(c, ensure(c->d_fwd_part, npart));
    if (want_loss) {
        StageScope sc(c, ST_MASK_SUM);
        HIPCHK(c, launch_mask_sum(mask, c->P, c->d_partial.p, c->d_msum.p, st));
    }
    unsigned long long* incut = nullptr;
    if (c->count_pairs) {
        HIPCHK(c, launch_fill_zero(c->d_incut.p, sizeof(unsigned long long), st));
        incut = c->d_incut.p;
    }
    {
        StageScope sc(c, ST_FORWARD);
        HIPCHK(c, launch_forward(ra, want_loss ? target : nullptr, mask, c->d_msum.p, pred, grad_pred,
                                 c->d_tile_sse.p, incut, c->d_work.p, npart ? c->d_fwd_part.p : nullptr, st));
    }
    if (want_loss) {
        StageScope sc(c, ST_LOSS);
        float* sse = slice_sse ? slice_sse : c->d_slice_sse.p;
        HIPCHK(c, launch_loss_finalize(c->d_tile_sse.p, c->d_geo.p, c->M,
                                       c->loss_kind == SVR_LOSS_MSE ? c->d_msum.p : nullptr, sse, loss, st));
    }
    if (c->check_flags & SVR_CHECK_FINITE) HIPCHK(c, launch_check_finite(pred, c->P, c->d_status.p, st));
    c->incut_pending = c->count_pairs;
    return SVR_OK;
}

int svr_backward(svr_ctx* c, const float* grad_pred, const float* grad_scale, const svr_grads* out) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!grad_pred) return fail(c, SVR_ERR_ARG, "grad_pred is NULL");
    if (!out || (c->N > 0 && (!out->mean || !out->log_scale || !out->quat || !out->amp)) ||
        (c->M > 0 && !out->pose))
        return fail(c, SVR_ERR_ARG, "a gradient output pointer is NULL");
    if (!c->binned) return fail(c, SVR_ERR_STATE, "svr_project_bin has not been called");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    hipStream_t st = c->stream;
    HIPCHK(c, ensure(c->d_work, 4));
    {
        StageScope sc(c, ST_ZERO);
        HIPCHK(c, launch_fill_zero(c->d_pose_acc.p, sizeof(float) * 6 * (size_t)c->M, st));
    }
    RenderArgs ra = render_args(c);
    {
        StageScope sc(c, ST_BACKWARD);
        HIPCHK(c, launch_backward(ra, grad_pred, grad_scale, c->d_inst_grad.p, c->d_work.p, st));
    }
    ProjectArgs pa = project_args(c);
    {
        StageScope sc(c, ST_PROJECT_BACKWARD);
        const bool two_level = c->max_subject_slices <= 512;
        if (two_level) {
            HIPCHK(c, ensure(c->d_pose_part, (size_t)std::max<int64_t>(c->pose_part_floats, 1)));
            HIPCHK(c, ensure(c->d_pose_pp, (size_t)std::max<int64_t>(c->pose_pp_floats, 1)));
        }
        HIPCHK(c, launch_project_backward(pa, c->d_offsets.p, c->d_counts.p, c->d_rec.p, c->d_rec_inst.p,
                                          c->d_inst_grad.p, c->n_inst, out->mean, out->log_scale, out->quat,
                                          out->amp, c->d_pose_acc.p, c->max_subject_slices,
                                          two_level ? c->d_pose_part.p : nullptr, two_level ? c->d_pose_pp.p : nullptr,
                                          c->d_pose_w1.p, c->n_pose_w1, c->d_pose_w2.p, c->n_pose_w2, c->M, st));
    }
    {
        StageScope sc(c, ST_POSE_CHAIN);
        HIPCHK(c, launch_pose_chain(c->params.pose, c->d_pose_acc.p, out->pose, c->M, st));
    }
    if (c->check_flags & SVR_CHECK_FINITE) {
        HIPCHK(c, launch_check_finite(out->mean, 3 * c->N, c->d_status.p, st));
        HIPCHK(c, launch_check_finite(out->log_scale, 3 * c->N, c->d_status.p, st));
        HIPCHK(c, launch_check_finite(out->quat, 4 * c->N, c->d_status.p, st));
        HIPCHK(c, launch_check_finite(out->amp, c->N, c->d_status.p, st));
        HIPCHK(c, launch_check_finite(out->pose, 6 * (int64_t)c->M, c->d_status.p, st));
    }
    return SVR_OK;
}

int svr_step(svr_ctx* c, const svr_grads* p, const svr_grads* g, float* m, float* v, const svr_adam* hp,
             int64_t step) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!p || !g || !hp || !m || !v) return fail(c, SVR_ERR_ARG, "NULL argument");
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "svr_set_geometry has not been called");
    if (step < 1) return fail(c, SVR_ERR_ARG, "step must be >= 1");
    if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0 && hp->beta2 >= 0.0 && hp->beta2 < 1.0 && hp->eps >= 0.0))
        return fail(c, SVR_ERR_ARG, "invalid Adam hyper-parameters");
    if (c->N > 0 && (!p->mean || !p->log_scale || !p->quat || !p->amp || !g->mean || !g->log_scale ||
                     !g->quat || !g->amp))
        return fail(c, SVR_ERR_ARG, "a parameter or gradient pointer is NULL");
    if (c->M > 0 && (!p->pose || !g->pose)) return fail(c, SVR_ERR_ARG, "pose pointer is NULL");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    const int64_t N = c->N, M = c->M;
    AdamSeg s[5];
    int ns = 0;
    int64_t off = 0;
    auto add = [&](float* pp, const float* gg, int64_t n, float la, float lb, int pose) {
        if (n <= 0) return;
        s[ns].p = pp;
        s[ns].g = gg;
        s[ns].n = n;
        s[ns].state_off = off;
        s[ns].lr_a = la;
        s[ns].lr_b = lb;
        s[ns].pose_layout = pose;
        ++ns;
    };
    add(p->mean, g->mean, 3 * N, hp->lr[0], hp->lr[0], 0); off += 3 * N;
    add(p->log_scale, g->log_scale, 3 * N, hp->lr[1], hp->lr[1], 0); off += 3 * N;
    add(p->quat, g->quat, 4 * N, hp->lr[2], hp->lr[2], 0); off += 4 * N;
    add(p->amp, g->amp, N, hp->lr[3], hp->lr[3], 0); off += N;
    add(p->pose, g->pose, 6 * M, hp->lr[4], hp->lr[5], 1);
    StageScope sc(c, ST_ADAM);
    HIPCHK(c, launch_adam(s, ns, m, v, hp->beta1, hp->beta2, hp->eps, hp->weight_decay, step, c->stream));
    return SVR_OK;
}

int svr_set_loss(svr_ctx* c, int kind) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (kind != SVR_LOSS_MSE && kind != SVR_LOSS_L1) return fail(c, SVR_ERR_ARG, "unknown loss kind %d", kind);
    c->loss_kind = kind;
    return SVR_OK;
}

int svr_scale_regularizer(svr_ctx* c, const float* log_scale, int64_t n, float lambda, float s_target,
                          float* g_log_scale, float* loss) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (n < 0) return fail(c, SVR_ERR_ARG, "n < 0");
    if (n > 0 && (!log_scale || !g_log_scale)) return fail(c, SVR_ERR_ARG, "log_scale or g_log_scale is NULL");
    if (!(lambda >= 0.f) || !isfinite(lambda) || !(s_target > 0.f) || !isfinite(s_target))
        return fail(c, SVR_ERR_ARG, "lambda must be finite and >= 0, s_target finite and > 0");
    if (n == 0) return SVR_OK;
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    HIPCHK(c, ensure(c->d_regpart, (size_t)kRegBlocks));
    HIPCHK(c, launch_scale_reg(log_scale, n, lambda, s_target, g_log_scale, loss, c->d_regpart.p, c->stream));
    return SVR_OK;
}

namespace {
// Uploads the per-slice and per-subject tables of the initialisation and runs
// the weight / cumulative-weight kernels into cdf [P]; copies the subjects'
// totals to host_total (synchronous).
int init_cdf(svr_ctx* c, const float* image, const float* mask, float lambda, int64_t* cdf,
             std::vector<int64_t>& host_total) {
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!image) return fail(c, SVR_ERR_ARG, "image is NULL");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(c, SVR_ERR_ARG, "lambda_init must be in [0, 1]");
    const int32_t S = c->n_subjects, M = c->M;
    std::vector<InitSlice> tab(M);
    int32_t max_hw = 1;
    for (int i = 0; i < M; ++i) {
        const double dx = c->spacing[2 * i], dy = c->spacing[2 * i + 1];
        tab[i].inv2_x = 0.5 / dx;
        tab[i].inv1_x = 1.0 / dx;
        tab[i].inv2_y = 0.5 / dy;
        tab[i].inv1_y = 1.0 / dy;
        tab[i].thick = c->fwhm[3 * i + 2];
        tab[i].pad = 0;
        max_hw = (int32_t)std::min<int64_t>(std::max<int64_t>(max_hw, (int64_t)c->H[i] * c->W[i]), 1 << 30);
    }
    std::vector<int64_t> sub_pix(S + 1, 0);
    {
        int i = 0;
        for (int s = 0; s < S; ++s) {
            sub_pix[s] = c->pix_off[i];
            while (i < M && c->slice_subject[i] == s) ++i;
        }
        sub_pix[S] = c->P;
    }
    hipStream_t st = c->stream;
    const int64_t nb = init_scan_blocks(c->P);
    HIPCHK(c, ensure(c->d_init_tab, (size_t)M));
    HIPCHK(c, ensure(c->d_init_subpix, (size_t)S + 1));
    HIPCHK(c, ensure(c->d_init_g, (size_t)c->P));
    HIPCHK(c, ensure(c->d_init_gmax, (size_t)S));
    HIPCHK(c, ensure(c->d_init_bsum, (size_t)nb));
    HIPCHK(c, ensure(c->d_init_base, (size_t)S));
    HIPCHK(c, ensure(c->d_init_total, (size_t)S));
    HIPCHK(c, hipMemcpyAsync(c->d_init_tab.p, tab.data(), tab.size() * sizeof(InitSlice), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->d_init_subpix.p, sub_pix.data(), sub_pix.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, st));
    HIPCHK(c, launch_init_cdf(c->d_geo.p, c->d_init_tab.p, M, max_hw, c->d_init_subpix.p, S, c->P, image, mask,
                              lambda, c->d_init_g.p, c->d_init_gmax.p, cdf, c->d_init_bsum.p, c->d_init_base.p,
                              c->d_init_total.p, st));
    host_total.assign(S, 0);
    HIPCHK(c, hipMemcpyAsync(host_total.data(), c->d_init_total.p, S * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return SVR_OK;
}
}  // namespace

int svr_init_cdf(svr_ctx* c, const float* image, const float* mask, float lambda_init, int64_t* cdf,
                 int64_t* totals) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!cdf) return fail(c, SVR_ERR_ARG, "cdf is NULL");
    std::vector<int64_t> tot;
    rc = init_cdf(c, image, mask, lambda_init, cdf, tot);
    if (rc != SVR_OK) return rc;
    if (totals) memcpy(totals, tot.data(), tot.size() * sizeof(int64_t));
    return SVR_OK;
}

int svr_init_means(svr_ctx* c, const float* image, const float* mask, const float* pose, float lambda_init,
                   const float* u, float* mean, int64_t* pixel, float* value) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (c->N == 0) return SVR_OK;
    if (!pose || !u || !mean) return fail(c, SVR_ERR_ARG, "pose, u or mean is NULL");
    if (((uintptr_t)u & 15) != 0) return fail(c, SVR_ERR_ARG, "u must be 16-byte aligned");
    HIPCHK(c, ensure(c->d_init_cdf, (size_t)c->P));
    std::vector<int64_t> tot;
    rc = init_cdf(c, image, mask, lambda_init, c->d_init_cdf.p, tot);
    if (rc != SVR_OK) return rc;
    for (int s = 0; s < c->n_subjects; ++s)
        if (c->gauss_off[s + 1] > c->gauss_off[s] && tot[s] <= 0)
            return fail(c, SVR_ERR_ARG, "subject %d has Gaussians but no pixel with positive weight", s);
    hipStream_t st = c->stream;
    HIPCHK(c, ensure(c->d_init_pose, (size_t)c->M));
    HIPCHK(c, launch_slice_pose(c->d_geo.p, pose, c->d_init_pose.p, c->M, st));
    HIPCHK(c, launch_init_sample(c->d_geo.p, c->d_init_pose.p, c->d_init_tab.p, c->d_subj.p, c->n_subjects,
                                 c->d_init_subpix.p, c->d_init_cdf.p, c->d_init_total.p, image, u, c->N, mean,
                                 pixel, value, st));
    return SVR_OK;
}

namespace {
int max_slice_pixels(const svr_ctx* c) {
    int64_t mx = 1;
    for (int i = 0; i < c->M; ++i) mx = std::max<int64_t>(mx, (int64_t)c->H[i] * c->W[i]);
    return (int)std::min<int64_t>(mx, 1 << 30);
}

int key_bits_for(int64_t n) {
    int kb = 1;
    while (kb < 32 && (1LL << kb) < n) ++kb;
    return kb;
}

int check_params(svr_ctx* c, const svr_params* p) {
    if (!p || (c->N > 0 && (!p->mean || !p->log_scale || !p->quat || !p->amp)) || (c->M > 0 && !p->pose))
        return fail(c, SVR_ERR_ARG, "a parameter pointer is NULL");
    return SVR_OK;
}
}  // namespace

int svr_topk_build(svr_ctx* c, const float* mean, const float* pose, const float* mask, int K, int32_t* nbr) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!mean || !pose || !nbr) return fail(c, SVR_ERR_ARG, "mean, pose or nbr is NULL");
    if (K < 1 || K > 1024) return fail(c, SVR_ERR_ARG, "K must be in [1, 1024]");
    if (c->M > 65535) return fail(c, SVR_ERR_CAPACITY, "more than 65535 slices");
    if ((int64_t)c->P * K > 0x7fffffffLL)
        return fail(c, SVR_ERR_CAPACITY, "P * K = %lld exceeds 2^31-1", (long long)c->P * K);
    const int32_t S = c->n_subjects, M = c->M;
    std::vector<int> has_slices(S, 0);
    for (int i = 0; i < M; ++i) has_slices[c->slice_subject[i]] = 1;
    for (int s = 0; s < S; ++s)
        if (has_slices[s] && c->gauss_off[s + 1] - c->gauss_off[s] < K)
            return fail(c, SVR_ERR_ARG, "subject %d has fewer than K = %d Gaussians", s, K);
    c->topk_built = false;
    c->topk_forwarded = false;
    hipStream_t st = c->stream;
    StageScope sc(c, ST_TOPK_KNN);
    HIPCHK(c, ensure(c->d_topk_pose, (size_t)M));
    HIPCHK(c, ensure(c->d_topk_slices, (size_t)M));
    HIPCHK(c, ensure(c->d_topk_bb, (size_t)6 * S));
    HIPCHK(c, ensure(c->d_topk_grid, (size_t)S));
    HIPCHK(c, ensure(c->d_topk_status, 2));
    HIPCHK(c, launch_slice_pose(c->d_geo.p, pose, c->d_topk_pose.p, M, st));
    HIPCHK(c, launch_topk_prepare(nullptr, nullptr, nullptr, nullptr, 0, nullptr, c->d_topk_pose.p, c->d_geo.p,
                                  nullptr, M, nullptr, c->d_topk_slices.p, st));
    HIPCHK(c, launch_topk_bbox(mean, c->d_blocks.p, c->n_blocks, S, c->d_topk_bb.p, st));
    std::vector<uint32_t> bb(6 * (size_t)S);
    HIPCHK(c, hipMemcpyAsync(bb.data(), c->d_topk_bb.p, bb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    // one cell grid per subject: about 8 means per cell on average
    std::vector<TopkGrid> grid(S);
    int64_t cells = 0;
    for (int s = 0; s < S; ++s) {
        TopkGrid& g = grid[s];
        memset(&g, 0, sizeof(g));
        const int64_t ns = c->gauss_off[s + 1] - c->gauss_off[s];
        double lo[3], ext[3], vol = 1.0;
        for (int d = 0; d < 3; ++d) {
            lo[d] = ns > 0 ? topk_order_float(bb[6 * s + d]) : 0.0;
            const double hi = ns > 0 ? topk_order_float(bb[6 * s + 3 + d]) : 0.0;
            ext[d] = std::max(hi - lo[d], 1e-3);
            vol *= ext[d];
        }
        double h = ns > 0 ? cbrt(vol / (double)ns * 8.0) : 1.0;
        h = std::max(h, 1e-3);
        int64_t dims[3];
        for (;;) {
            for (int d = 0; d < 3; ++d) dims[d] = (int64_t)floor(ext[d] / h) + 1;
            if (dims[0] * dims[1] * dims[2] <= (1LL << 24)) break;
            h *= 1.25;
        }
        for (int d = 0; d < 3; ++d) {
            g.origin[d] = (float)lo[d];
            g.dims[d] = (int32_t)dims[d];
        }
        g.h = (float)h;
        g.inv_h = (float)(1.0 / h);
        // radius holding about K means at the subject's mean density, with margin
        const double dens = ns > 0 ? (double)ns / vol : 1.0;
        g.rho0 = (float)(1.3 * cbrt(3.0 * K / (4.0 * M_PI * dens)));
        g.base = cells;
        cells += dims[0] * dims[1] * dims[2];
    }
    if (cells > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "neighbour grid too large");
    HIPCHK(c, hipMemcpyAsync(c->d_topk_grid.p, grid.data(), grid.size() * sizeof(TopkGrid), hipMemcpyHostToDevice, st));
    const int64_t N = c->N;
    HIPCHK(c, ensure(c->d_topk_cells, (size_t)cells));
    HIPCHK(c, ensure(c->d_topk_smean, (size_t)N));
    HIPCHK(c, ensure(c->d_topk_ck, (size_t)N));
    HIPCHK(c, ensure(c->d_topk_cv, (size_t)N));
    HIPCHK(c, ensure(c->d_topk_ck2, (size_t)N));
    HIPCHK(c, ensure(c->d_topk_cv2, (size_t)N));
    const int64_t n_pairs = c->P * (int64_t)K;
    HIPCHK(c, ensure(c->d_topk_sort_tmp, std::max(sort_tmp_bytes(N), sort_tmp_bytes(n_pairs))));   // n_act*K <= n_pairs
    HIPCHK(c, launch_topk_cells(mean, c->d_blocks.p, c->n_blocks, c->d_topk_grid.p, N, cells, c->d_topk_ck.p,
                                c->d_topk_cv.p, c->d_topk_ck2.p, c->d_topk_cv2.p, c->d_topk_sort_tmp.p,
                                key_bits_for(cells), c->d_topk_cells.p, c->d_topk_smean.p, &c->topk_perm, st));
    int max_tiles = 1;
    for (int i = 0; i < M; ++i) max_tiles = std::max(max_tiles, topk_knn_tiles(c->H[i], c->W[i]));
    HIPCHK(c, launch_fill_zero(c->d_topk_status.p, 2 * sizeof(int), st));
    HIPCHK(c, launch_topk_knn(c->d_geo.p, c->d_topk_slices.p, c->d_topk_grid.p, c->d_topk_cells.p,
                              c->d_topk_smean.p, mask, M, max_tiles, K, nbr, c->d_topk_status.p, st));
    int status[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(status, c->d_topk_status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->topk_split_tiles = status[1];
    if (status[0] > 0)
        return fail(c, SVR_ERR_CAPACITY, "neighbour search failed for %d pixels (too dense or too far from the means)",
                    status[0]);
    {
        StageScope sc2(c, ST_TOPK_INVERSE);
        // the pixels with a list, per slice
        const int64_t P = c->P;
        std::vector<int64_t> qoff(M + 1, 0);
        for (int i = 0; i < M; ++i)
            qoff[i + 1] = qoff[i] + (int64_t)((c->H[i] + 7) / 8 * 8) * ((c->W[i] + 7) / 8 * 8);
        const int64_t Q = qoff[M];
        if (Q > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "too many pixels for the neighbour lists");
        HIPCHK(c, ensure(c->d_topk_qoff, (size_t)M + 1));
        HIPCHK(c, hipMemcpyAsync(c->d_topk_qoff.p, qoff.data(), qoff.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                                 st));
        HIPCHK(c, ensure(c->d_topk_flag, (size_t)Q));
        HIPCHK(c, ensure(c->d_topk_aoff, (size_t)Q));
        HIPCHK(c, ensure(c->d_topk_active, (size_t)P));
        HIPCHK(c, ensure(c->d_topk_act, (size_t)P));
        HIPCHK(c, ensure(c->d_topk_act_off, (size_t)M + 1));
        HIPCHK(c, ensure(c->d_topk_scan_tmp, scan_tmp_bytes(Q)));
        HIPCHK(c, ensure(c->d_topk_tot, 2));
        HIPCHK(c, launch_topk_active(nbr, K, c->d_geo.p, c->d_topk_qoff.p, M, Q, c->d_topk_flag.p, c->d_topk_aoff.p,
                                     c->d_topk_active.p, c->d_topk_act.p, c->d_topk_act_off.p, c->d_topk_tot.p,
                                     c->d_topk_scan_tmp.p, st));
        std::vector<int32_t> aoff(M + 1);
        HIPCHK(c, hipMemcpyAsync(aoff.data(), c->d_topk_act_off.p, aoff.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        c->topk_n_act = aoff[M];
        c->topk_max_act = 1;
        for (int i = 0; i < M; ++i) c->topk_max_act = std::max(c->topk_max_act, aoff[i + 1] - aoff[i]);
        // internal lists (cell-order positions) and their inverse
        const int64_t n_int = c->topk_n_act * (int64_t)K;
        HIPCHK(c, ensure(c->d_topk_iperm, (size_t)N));
        HIPCHK(c, ensure(c->d_topk_lint, (size_t)n_int));
        HIPCHK(c, launch_topk_internal(nbr, c->d_topk_act.p, c->topk_n_act, K, c->topk_perm, N, c->d_topk_iperm.p,
                                       c->d_topk_lint.p, st));
        HIPCHK(c, ensure(c->d_topk_pk, (size_t)n_int));
        HIPCHK(c, ensure(c->d_topk_pv, (size_t)n_int));
        HIPCHK(c, ensure(c->d_topk_pk2, (size_t)n_int));
        HIPCHK(c, ensure(c->d_topk_pv2, (size_t)n_int));
        HIPCHK(c, ensure(c->d_topk_granges, (size_t)N));
        HIPCHK(c, launch_topk_inverse(c->d_topk_lint.p, n_int, N, key_bits_for(N), c->d_topk_pk.p, c->d_topk_pv.p,
                                      c->d_topk_pk2.p, c->d_topk_pv2.p, c->d_topk_sort_tmp.p, c->d_topk_granges.p,
                                      &c->topk_gpix, st));
    }
    c->topk_nbr = nbr;
    c->topk_K = K;
    c->topk_built = true;
    return SVR_OK;
}

int svr_topk_forward(svr_ctx* c, const svr_params* params, const float* sigma, const int32_t* nbr, int K,
                     float delta, const float* target, const float* mask, float* pred, float* loss,
                     float* grad_pred) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!pred) return fail(c, SVR_ERR_ARG, "pred is NULL");
    if ((rc = check_params(c, params)) != SVR_OK) return rc;
    const bool want_loss = loss || grad_pred;
    if (want_loss && (!target || !mask))
        return fail(c, SVR_ERR_ARG, "loss outputs requested without target and mask");
    if (!(delta > 0.f) || !isfinite(delta)) return fail(c, SVR_ERR_ARG, "delta must be finite and > 0");
    if (!c->topk_built || nbr != c->topk_nbr || K != c->topk_K)
        return fail(c, SVR_ERR_STATE, "nbr / K are not those of the last svr_topk_build");
    hipStream_t st = c->stream;
    const int32_t M = c->M;
    const int mhw = max_slice_pixels(c);
    HIPCHK(c, ensure(c->d_topk_gauss, (size_t)c->N));
    HIPCHK(c, ensure(c->d_topk_state, (size_t)std::max<int64_t>(c->topk_n_act, 1)));
    HIPCHK(c, ensure(c->d_topk_partial, std::max(std::max(topk_pose_partial_floats(M, c->topk_max_act),
                                                          topk_loss_partial_floats(M, mhw, c->topk_max_act)),
                                                 (size_t)1024)));
    HIPCHK(c, ensure(c->d_topk_msum, 1));
    HIPCHK(c, ensure(c->d_partial, 1024));
    StageScope sc(c, ST_TOPK_FORWARD);
    HIPCHK(c, launch_slice_pose(c->d_geo.p, params->pose, c->d_topk_pose.p, M, st));
    HIPCHK(c, launch_topk_prepare(params->mean, params->log_scale, params->quat, params->amp, c->N, c->topk_perm,
                                  c->d_topk_pose.p, c->d_geo.p, sigma, M, c->d_topk_gauss.p, c->d_topk_slices.p, st));
    if (want_loss && c->loss_kind == SVR_LOSS_MSE)
        HIPCHK(c, launch_mask_sum(mask, c->P, c->d_partial.p, c->d_topk_msum.p, st));
    HIPCHK(c, launch_topk_forward(c->d_geo.p, c->d_topk_slices.p, c->d_topk_gauss.p, c->d_topk_lint.p, c->d_topk_act.p,
                                  c->d_topk_act_off.p, c->d_topk_active.p, c->topk_n_act, K, delta, c->loss_kind, M, mhw,
                                  c->topk_max_act, want_loss ? target : nullptr, mask,
                                  c->loss_kind == SVR_LOSS_MSE ? c->d_topk_msum.p : nullptr, pred,
                                  c->d_topk_state.p, grad_pred, c->d_topk_partial.p, loss, st));
    c->topk_forwarded = true;
    return SVR_OK;
}

int svr_topk_backward(svr_ctx* c, const svr_params* params, const int32_t* nbr, int K, const float* grad_pred,
                      const svr_grads* out, float* g_sigma) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if ((rc = check_params(c, params)) != SVR_OK) return rc;
    if (!grad_pred) return fail(c, SVR_ERR_ARG, "grad_pred is NULL");
    if (!out || (c->N > 0 && (!out->mean || !out->log_scale || !out->quat || !out->amp)) ||
        (c->M > 0 && !out->pose))
        return fail(c, SVR_ERR_ARG, "a gradient output pointer is NULL");
    if (!c->topk_built || nbr != c->topk_nbr || K != c->topk_K)
        return fail(c, SVR_ERR_STATE, "nbr / K are not those of the last svr_topk_build");
    if (!c->topk_forwarded) return fail(c, SVR_ERR_STATE, "svr_topk_forward has not been called");
    hipStream_t st = c->stream;
    const int32_t M = c->M;
    const int mhw = max_slice_pixels(c);
    HIPCHK(c, ensure(c->d_topk_pose_acc, (size_t)6 * std::max(M, 1)));
    HIPCHK(c, ensure(c->d_topk_pxw, (size_t)std::max<int64_t>(c->topk_n_act, 1)));
    HIPCHK(c, ensure(c->d_topk_pyd, (size_t)std::max<int64_t>(c->topk_n_act, 1)));
    (void)mhw;
    StageScope sc(c, ST_TOPK_BACKWARD);
    HIPCHK(c, launch_topk_backward(c->d_geo.p, c->d_topk_slices.p, c->d_topk_gauss.p, c->d_topk_lint.p, c->d_topk_act.p,
                                   c->d_topk_act_off.p, c->topk_n_act, K, M, c->topk_max_act,
                                   grad_pred, c->d_topk_state.p, c->d_topk_granges.p, c->topk_gpix, c->topk_perm,
                                   params->log_scale, params->quat, c->N, out->mean, out->log_scale, out->quat,
                                   out->amp, c->d_topk_partial.p, c->d_topk_pose_acc.p, g_sigma, c->d_topk_pxw.p,
                                   c->d_topk_pyd.p, st));
    HIPCHK(c, launch_pose_chain(params->pose, c->d_topk_pose_acc.p, out->pose, M, st));
    return SVR_OK;
}

int svr_slice_loss(svr_ctx* c, const float* pred, const float* target, const float* mask, const float* sigma,
                   const float* log_omega, float* loss, float* grad_pred, float* slice_sums, float* g_sigma,
                   float* g_log_omega) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!pred || !target || !mask) return fail(c, SVR_ERR_ARG, "pred, target or mask is NULL");
    hipStream_t st = c->stream;
    const int mhw = max_slice_pixels(c);
    HIPCHK(c, ensure(c->d_sl_scratch, slice_loss_partial_floats(std::max(c->M, 1), mhw, c->n_subjects)));
    HIPCHK(c, ensure(c->d_sl_msum, 1));
    HIPCHK(c, ensure(c->d_partial, 1024));
    if (c->loss_kind == SVR_LOSS_MSE) HIPCHK(c, launch_mask_sum(mask, c->P, c->d_partial.p, c->d_sl_msum.p, st));
    else HIPCHK(c, launch_fill_zero(c->d_sl_msum.p, sizeof(float), st));
    HIPCHK(c, launch_slice_loss(c->d_geo.p, c->d_subj.p, c->n_subjects, c->M, mhw, pred, target, mask, sigma,
                                log_omega, c->d_sl_msum.p, c->loss_kind, loss, grad_pred, slice_sums, g_sigma,
                                g_log_omega, c->d_sl_scratch.p, st));
    return SVR_OK;
}

int svr_bias_apply(svr_ctx* c, const float* centres, float width, const float* beta, int32_t K, float* pred,
                   float* bias) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!c->binned) return fail(c, SVR_ERR_STATE, "svr_project_bin has not been called");
    if (!centres || !beta || !pred) return fail(c, SVR_ERR_ARG, "centres, beta or pred is NULL");
    if (K < 1 || K > SVR_BIAS_MAX_K) return fail(c, SVR_ERR_ARG, "K = %d outside [1, %d]", K, SVR_BIAS_MAX_K);
    if (!(width > 0.f) || !(width < 3.0e38f)) return fail(c, SVR_ERR_ARG, "width must be positive and finite");
    HIPCHK(c, launch_bias_apply(c->d_geo.p, c->d_pose.p, c->M, max_slice_pixels(c), centres, width, beta, K, pred,
                                bias, c->stream));
    return SVR_OK;
}

int svr_bias_backward(svr_ctx* c, const float* centres, float width, const float* beta, int32_t K,
                      const float* pred_biased, const float* bias, float* grad_pred, float* g_beta, float* g_pose) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!c->binned) return fail(c, SVR_ERR_STATE, "svr_project_bin has not been called");
    if (!centres || !beta || !pred_biased || !bias || !grad_pred || !g_beta)
        return fail(c, SVR_ERR_ARG, "NULL argument");
    if (K < 1 || K > SVR_BIAS_MAX_K) return fail(c, SVR_ERR_ARG, "K = %d outside [1, %d]", K, SVR_BIAS_MAX_K);
    if (!(width > 0.f) || !(width < 3.0e38f)) return fail(c, SVR_ERR_ARG, "width must be positive and finite");
    const int mhw = max_slice_pixels(c);
    HIPCHK(c, ensure(c->d_bias_scratch, bias_scratch_floats(std::max(c->M, 1), mhw, K)));
    HIPCHK(c, launch_bias_backward(c->d_geo.p, c->d_pose.p, c->d_subj.p, c->n_subjects, c->M, mhw, centres, width,
                                   beta, K, pred_biased, bias, grad_pred, g_beta, g_pose,
                                   c->d_bias_scratch.p, c->stream));
    return SVR_OK;
}

int svr_densify_accumulate(svr_ctx* c, const float* g_mean, float* grad_acc, int32_t* count) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (c->N == 0) return SVR_OK;
    if (!g_mean || !grad_acc || !count) return fail(c, SVR_ERR_ARG, "g_mean, grad_acc or count is NULL");
    HIPCHK(c, launch_densify_accumulate(g_mean, grad_acc, count, c->N, c->stream));
    return SVR_OK;
}

int svr_densify(svr_ctx* c, const svr_params* in, const float* grad_acc, const int32_t* count,
                const svr_densify_cfg* cfg, const svr_grads* out, int64_t capacity, int32_t* src,
                const float* exp_avg_in, const float* exp_avg_sq_in, float* exp_avg_out, float* exp_avg_sq_out,
                int64_t* new_offsets) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "no geometry set");
    if (!in || !cfg || !out || !new_offsets) return fail(c, SVR_ERR_ARG, "in, cfg, out or new_offsets is NULL");
    const int64_t N = c->N;
    if (N > 0 && (!in->mean || !in->log_scale || !in->quat || !in->amp || !grad_acc || !count))
        return fail(c, SVR_ERR_ARG, "an input array is NULL");
    if (!(cfg->split_offset > 0.f && cfg->split_offset < 1.f))
        return fail(c, SVR_ERR_ARG, "split_offset must lie in (0, 1)");
    if (!(cfg->clone_offset >= 0.f) || !isfinite(cfg->clone_offset))
        return fail(c, SVR_ERR_ARG, "clone_offset must be >= 0 and finite");
    if (!(cfg->grad_threshold >= 0.f) || isnan(cfg->log_scale_threshold) || isnan(cfg->prune_amp))
        return fail(c, SVR_ERR_ARG, "grad_threshold must be >= 0; thresholds must not be NaN");
    const bool moments = exp_avg_in || exp_avg_sq_in || exp_avg_out || exp_avg_sq_out;
    if (moments && !(exp_avg_in && exp_avg_sq_in && exp_avg_out && exp_avg_sq_out))
        return fail(c, SVR_ERR_ARG, "the four moment arrays are given together or not at all");
    if (moments && (exp_avg_out == exp_avg_in || exp_avg_sq_out == exp_avg_sq_in))
        return fail(c, SVR_ERR_ARG, "moments cannot be remapped in place");
    if (2 * N > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "2 N exceeds 2^31-1");
    hipStream_t st = c->stream;
    const int S = c->n_subjects;
    HIPCHK(c, ensure(c->d_dens_n, (size_t)N));
    HIPCHK(c, ensure(c->d_dens_pos, (size_t)N));
    HIPCHK(c, ensure(c->d_dens_off, (size_t)S + 1));
    HIPCHK(c, ensure(c->d_dens_tot, 2));
    HIPCHK(c, ensure(c->d_scan_tmp, scan_tmp_bytes(N) + 64));
    HIPCHK(c, launch_densify_plan(grad_acc, count, in->amp, N, cfg->grad_threshold, cfg->prune_amp, c->d_subj.p, S,
                                  c->d_dens_n.p, c->d_dens_pos.p, c->d_dens_tot.p, c->d_scan_tmp.p, c->d_dens_off.p,
                                  st));
    std::vector<int64_t> off((size_t)S + 1);
    HIPCHK(c, hipMemcpyAsync(off.data(), c->d_dens_off.p, sizeof(int64_t) * (S + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int s = 0; s <= S; ++s) new_offsets[s] = off[s];
    const int64_t K = off[S];
    if (K > capacity)
        return fail(c, SVR_ERR_CAPACITY, "densified mixture has %lld Gaussians, capacity %lld", (long long)K,
                    (long long)capacity);
    if (K > 0 && (!out->mean || !out->log_scale || !out->quat || !out->amp))
        return fail(c, SVR_ERR_ARG, "an output array is NULL");
    const double a = cfg->split_offset;
    DensifyArgs d;
    d.mean = in->mean; d.log_scale = in->log_scale; d.quat = in->quat; d.amp = in->amp;
    d.n_out = c->d_dens_n.p; d.pos = c->d_dens_pos.p;
    d.n = N; d.n_new = K;
    d.o_mean = out->mean; d.o_log_scale = out->log_scale; d.o_quat = out->quat; d.o_amp = out->amp;
    d.src = src;
    d.m1_in = exp_avg_in; d.m2_in = exp_avg_sq_in; d.m1_out = exp_avg_out; d.m2_out = exp_avg_sq_out;
    d.log_scale_thr = cfg->log_scale_threshold;
    d.split_offset = cfg->split_offset;
    d.clone_offset = cfg->clone_offset;
    d.split_dlog = (float)(0.5 * std::log1p(-a * a));
    d.split_amp = (float)(0.5 / std::sqrt(1.0 - a * a));
    HIPCHK(c, launch_densify_emit(d, st));
    if (moments && c->M > 0) {
        HIPCHK(c, hipMemcpyAsync(exp_avg_out + 11 * K, exp_avg_in + 11 * N, sizeof(float) * 6 * (size_t)c->M,
                                 hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(exp_avg_sq_out + 11 * K, exp_avg_sq_in + 11 * N, sizeof(float) * 6 * (size_t)c->M,
                                 hipMemcpyDeviceToDevice, st));
    }
    // the context now describes the densified mixture
    c->gauss_off.assign(off.begin(), off.end());
    c->N = K;
    c->topk_built = false;
    c->topk_forwarded = false;
    return build_tables(c);
}

int svr_adam_vector(svr_ctx* c, float* p, const float* g, float* exp_avg, float* exp_avg_sq, int64_t n, float lr,
                    const svr_adam* hp, int64_t step) {
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (n < 0) return fail(c, SVR_ERR_ARG, "n < 0");
    if (n == 0) return SVR_OK;
    if (!p || !g || !exp_avg || !exp_avg_sq || !hp) return fail(c, SVR_ERR_ARG, "NULL argument");
    if (step < 1) return fail(c, SVR_ERR_ARG, "step must be >= 1");
    if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0 && hp->beta2 >= 0.0 && hp->beta2 < 1.0 && hp->eps >= 0.0))
        return fail(c, SVR_ERR_ARG, "invalid Adam hyper-parameters");
    AdamSeg s;
    s.p = p;
    s.g = g;
    s.n = n;
    s.state_off = 0;
    s.lr_a = s.lr_b = lr;
    s.pose_layout = 0;
    HIPCHK(c, launch_adam(&s, 1, exp_avg, exp_avg_sq, hp->beta1, hp->beta2, hp->eps, hp->weight_decay, step,
                          c->stream));
    return SVR_OK;
}

int svr_set_count_pairs(svr_ctx* c, int enable) {
    if (!c) return SVR_ERR_ARG;
    c->count_pairs = enable != 0;
    return SVR_OK;
}

int svr_get_stats(svr_ctx* c, int flags, svr_stats* out) {
    if (!c || !out) return SVR_ERR_ARG;
    c->err.clear();
    memset(out, 0, sizeof(*out));
    out->n_gauss = c->N;
    out->n_slices = c->M;
    out->n_pixels = c->P;
    out->n_tiles = c->n_tiles;
    out->key_bits = c->key_bits;
    {
        const int sb = c->key_bits - kClassBits, dw = radix_digit_bits(sb);
        out->sort_passes = (sb + dw - 1) / dw;
    }
    out->n_candidates = c->binned ? c->n_cand : 0;
    out->n_records = c->binned ? c->n_rec : 0;
    out->n_instances = c->binned ? c->n_inst : 0;
    out->n_incut = -1;
    out->n_evaluated = -1;
    if (c->binned) {
        // evaluated pixel-record terms of the forward: every instance costs a
        // full tile of pixels (before per-wave row culling)
        out->n_evaluated = c->n_inst * (int64_t)c->cfg.tile * c->cfg.tile;
    }
    out->n_fallback_blocks = -1;
    const bool fixed = c->cap_rec > 0;
    if (fixed && c->binned) {  // the host holds only the capacity
        out->n_records = -1;
        out->n_instances = -1;
        out->n_evaluated = -1;
    }
    if ((flags & SVR_STATS_SYNC) && !c->host_only) {
        int rc = enter(c);
        if (rc != SVR_OK) return rc;
        if (c->incut_pending) {
            unsigned long long h = 0;
            HIPCHK(c, hipMemcpyAsync(&h, c->d_incut.p, sizeof h, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            c->n_incut = (int64_t)h;
            c->incut_pending = false;
        }
        if (c->binned) {
            std::vector<int> fb((size_t)std::max(c->n_blocks, 0));
            if (!fb.empty())
                HIPCHK(c, hipMemcpyAsync(fb.data(), c->d_fallback.p, fb.size() * sizeof(int), hipMemcpyDeviceToHost,
                                         c->stream));
            long long tot[2] = {0, 0};
            if (fixed) HIPCHK(c, hipMemcpyAsync(tot, c->d_totals.p, sizeof tot, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            int64_t nf = 0;
            for (int v : fb) nf += v != 0;
            out->n_fallback_blocks = nf;
            if (fixed) {
                out->n_records = tot[0];
                out->n_instances = tot[1];
                out->n_evaluated = tot[1] * (int64_t)c->cfg.tile * c->cfg.tile;
            }
        }
    }
    out->n_incut = c->n_incut;
    return SVR_OK;
}

int svr_set_capacity(svr_ctx* c, int64_t max_records, int64_t max_instances) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (max_records < 0 || max_instances < 0 || ((max_records == 0) != (max_instances == 0)))
        return fail(c, SVR_ERR_ARG, "capacities must both be positive, or both 0 (got %lld, %lld)",
                    (long long)max_records, (long long)max_instances);
    if (max_records > 0x7fffffffLL || max_instances > 0x7fffffffLL)
        return fail(c, SVR_ERR_CAPACITY, "capacities above 2^31-1");
    c->binned = false;
    c->cap_rec = max_records;
    c->cap_inst = max_instances;
    if (max_records == 0 || c->host_only) return SVR_OK;
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    rc = ensure_bin_buffers(c, max_records, max_instances);
    if (rc != SVR_OK) {
        c->cap_rec = c->cap_inst = 0;
        return rc;
    }
    return SVR_OK;
}

int svr_set_checks(svr_ctx* c, int flags) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (flags & ~SVR_CHECK_FINITE) return fail(c, SVR_ERR_ARG, "unknown check flags 0x%x", flags);
    c->check_flags = flags;
    return SVR_OK;
}

int svr_check_status(svr_ctx* c, int64_t* needed_records, int64_t* needed_instances) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (needed_records) *needed_records = 0;
    if (needed_instances) *needed_instances = 0;
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    HIPCHK(c, hipMemcpyAsync(c->h_status, c->d_status.p, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const DevStatus h = *c->h_status;
    if (h.bits == 0) return SVR_OK;
    // clear the recorded conditions (the overflow flag of the last binning stays)
    HIPCHK(c, launch_fill_zero(&c->d_status.p->bits, sizeof(unsigned int), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.bits & kStatusCapacity) {
        if (needed_records) *needed_records = h.need_rec;
        if (needed_instances) *needed_instances = h.need_inst;
        return fail(c, SVR_ERR_CAPACITY, "a fixed-capacity binning needed %lld records and %lld instances",
                    (long long)h.need_rec, (long long)h.need_inst);
    }
    return fail(c, SVR_ERR_NONFINITE, "a checked parameter, prediction or gradient was NaN or infinite");
}

int svr_set_timing(svr_ctx* c, int enable) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        int rc = fold_timing(c);
        if (rc != SVR_OK) return rc;
    }
    c->timing = enable != 0;
    for (int s = 0; s < ST_COUNT; ++s) {
        c->t_ms[s] = 0.0;
        c->t_calls[s] = 0;
    }
    return SVR_OK;
}

int svr_set_timing_stages(svr_ctx* c, uint32_t mask) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    c->timing_mask = mask;
    return SVR_OK;
}

int svr_get_timing(svr_ctx* c, svr_timer* out, int max_out, int* n_out) {
    if (!c || (max_out > 0 && !out)) return SVR_ERR_ARG;
    c->err.clear();
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        int rc = fold_timing(c);
        if (rc != SVR_OK) return rc;
    }
    int n = 0;
    for (int s = 0; s < ST_COUNT && n < max_out; ++s, ++n) {
        memset(out[n].name, 0, sizeof out[n].name);
        strncpy(out[n].name, kStageNames[s], sizeof out[n].name - 1);
        out[n].calls = c->t_calls[s];
        out[n].total_ms = c->t_ms[s];
    }
    if (n_out) *n_out = n;
    return SVR_OK;
}

int svr_sort_pairs(svr_ctx* c, uint32_t* keys, uint32_t* vals, int64_t n, int key_bits) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (n < 0 || key_bits < 1 || key_bits > 32) return fail(c, SVR_ERR_ARG, "n < 0 or key_bits out of range");
    if (n > 0 && (!keys || !vals)) return fail(c, SVR_ERR_ARG, "keys/vals NULL");
    if (n > 0x7fffffffLL) return fail(c, SVR_ERR_CAPACITY, "n exceeds 2^31-1");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (n <= 1) return SVR_OK;
    hipStream_t st = c->stream;
    DevBuf<uint32_t> k2, v2;
    DevBuf<char> tmp;
    HIPCHK(c, ensure(k2, (size_t)n, true));
    HIPCHK(c, ensure(v2, (size_t)n, true));
    HIPCHK(c, ensure(tmp, sort_tmp_bytes(n), true));
    bool alt = false;
    hipError_t e = launch_radix_sort(keys, vals, k2.p, v2.p, n, key_bits, tmp.p, &alt, st);
    if (e == hipSuccess && alt) {
        e = hipMemcpyAsync(keys, k2.p, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(vals, v2.p, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    }
    hipError_t e2 = hipStreamSynchronize(st);
    release(k2);
    release(v2);
    release(tmp);
    if (e != hipSuccess) return fail(c, SVR_ERR_HIP, "radix sort: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(c, SVR_ERR_HIP, "radix sort sync: %s", hipGetErrorString(e2));
    return SVR_OK;
}

int svr_sort_pairs_noalloc(svr_ctx* c, uint32_t* keys, uint32_t* vals, int64_t n, int key_bits) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (n < 0 || key_bits < 1 || key_bits > 32) return fail(c, SVR_ERR_ARG, "n < 0 or key_bits out of range");
    if (n > 0 && (!keys || !vals)) return fail(c, SVR_ERR_ARG, "keys/vals NULL");
    if (n > kNoallocMax)
        return fail(c, SVR_ERR_CAPACITY, "n = %lld exceeds the allocation-free maximum %lld", (long long)n,
                    (long long)kNoallocMax);
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    if (n <= 1) return SVR_OK;
    if (sort_tmp_bytes(n) > kNoallocTmp) return fail(c, SVR_ERR_CAPACITY, "sort scratch exceeds its reserve");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (c->device >= kNoallocDevices || !g_noalloc_done[c->device])
            return fail(c, SVR_ERR_STATE, "no scratch address for device %d", c->device);
        if (g_noalloc_err[c->device] != hipSuccess)
            return fail(c, SVR_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(g_noalloc_err[c->device]));
        base = g_noalloc_ptr[c->device];
    }
    uint32_t* k2 = (uint32_t*)base;
    uint32_t* v2 = k2 + kNoallocMax;
    void* tmp = (char*)base + 2 * kNoallocKV;
    hipStream_t st = c->stream;
    bool alt = false;
    hipError_t e = launch_radix_sort(keys, vals, k2, v2, n, key_bits, tmp, &alt, st);
    if (e == hipSuccess && alt) {
        e = hipMemcpyAsync(keys, k2, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(vals, v2, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) return fail(c, SVR_ERR_HIP, "radix sort: %s", hipGetErrorString(e));
    return SVR_OK;
}


static std::string tune_key(const svr_ctx* c) {
    auto lg = [](int64_t v) {
        int k = 0;
        while (v > 1) { v >>= 1; ++k; }
        return k;
    };
    // only quantities that do not depend on the configuration (the instance
    // count changes with the tile size, so a key holding it would miss once
    // the tuned tile size is installed)
    char buf[128];
    snprintf(buf, sizeof buf, "gfx950:P%d:R%d:S%d", lg(c->P), lg(c->n_rec), c->n_subjects);
    return buf;
}

static void tune_cache_load(svr_ctx* c, const char* path) {
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[128];
    svr_config g;
    while (fscanf(f, "%127s %d %d %d %f %d", key, &g.tile, &g.batch, &g.persistent, &g.cutoff, &g.forward_mode) == 6)
        if (valid_config(g)) c->tune_cache[key] = g;
    fclose(f);
}

static void tune_cache_save(svr_ctx* c, const char* path) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto& kv : c->tune_cache)
        fprintf(f, "%s %d %d %d %.6g %d\n", kv.first.c_str(), kv.second.tile, kv.second.batch, kv.second.persistent,
                (double)kv.second.cutoff, kv.second.forward_mode);
    fclose(f);
    rename(tmp.c_str(), path);
}

int svr_autotune(svr_ctx* c, const svr_params* params, const float* grad_pred, int flags, const char* cache_path,
                 svr_config* out, float* times_ms, int max_times) {
    if (!c) return SVR_ERR_ARG;
    c->err.clear();
    if (!params || !grad_pred || !out) return fail(c, SVR_ERR_ARG, "NULL argument");
    if (!c->has_geom) return fail(c, SVR_ERR_STATE, "svr_set_geometry has not been called");
    int rc = enter(c);
    if (rc != SVR_OK) return rc;
    hipStream_t st = c->stream;
    const svr_config base = c->cfg;
    if (!c->binned || c->params.mean != params->mean) {
        rc = project_bin_impl(c, params);
        if (rc != SVR_OK) return rc;
    }
    tune_cache_load(c, cache_path);
    const std::string key = tune_key(c);
    auto hit = c->tune_cache.find(key);
    if (hit != c->tune_cache.end()) {
        svr_config g = hit->second;
        g.cutoff = base.cutoff;
        rc = svr_set_config(c, &g);
        if (rc != SVR_OK) return rc;
        if (!c->binned) {
            rc = project_bin_impl(c, params);
            if (rc != SVR_OK) return rc;
        }
        *out = c->cfg;
        return SVR_OK;
    }
    DevBuf<float> pred, grads;
    HIPCHK(c, ensure(pred, (size_t)c->P, true));
    const size_t ng = (size_t)c->N * 11 + (size_t)c->M * 6;
    HIPCHK(c, ensure(grads, ng, true));
    svr_grads gout;
    gout.mean = grads.p;
    gout.log_scale = grads.p + 3 * c->N;
    gout.quat = grads.p + 6 * c->N;
    gout.amp = grads.p + 10 * c->N;
    gout.pose = grads.p + 11 * c->N;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    std::vector<int> tiles = (flags & SVR_TUNE_TILE) ? std::vector<int>{8, 16, 32} : std::vector<int>{base.tile};
    std::vector<int> batches =
        (flags & SVR_TUNE_BATCH) ? std::vector<int>{32, 64, 128, 256} : std::vector<int>{base.batch};
    std::vector<int> pers = (flags & SVR_TUNE_PERSISTENT) ? std::vector<int>{0, 1} : std::vector<int>{base.persistent};
    std::vector<int> modes = (flags & SVR_TUNE_MODE) ? std::vector<int>{0, 1, 2} : std::vector<int>{base.forward_mode};
    float best = 1e30f;
    svr_config best_cfg = base;
    int nt = 0;
    int status = SVR_OK;
    for (int T : tiles) {
        for (int P : pers) {
            svr_config g = base;
            g.tile = T;
            g.persistent = P;
            status = svr_set_config(c, &g);
            if (status != SVR_OK) break;
            // binning depends on the tile size (instances, key bits, sort
            // passes): its time counts toward every configuration of this tile
            float bin_ms = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                if (hipEventRecord(e0, st) != hipSuccess) { status = SVR_ERR_HIP; break; }
                status = project_bin_impl(c, params);
                if (status != SVR_OK) break;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    status = SVR_ERR_HIP;
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                bin_ms = std::min(bin_ms, ms);
            }
            if (status != SVR_OK) break;
            for (int FM : modes)
            for (int B : (FM == 0 ? batches : std::vector<int>{base.batch})) {
                c->cfg.batch = B;
                c->cfg.forward_mode = FM;
                float tbest = 1e30f;
                for (int rep = 0; rep < 4; ++rep) {
                    if (hipEventRecord(e0, st) != hipSuccess) { status = SVR_ERR_HIP; break; }
                    status = svr_forward(c, nullptr, nullptr, pred.p, nullptr, nullptr, nullptr);
                    if (status != SVR_OK) break;
                    status = svr_backward(c, grad_pred, nullptr, &gout);
                    if (status != SVR_OK) break;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        status = SVR_ERR_HIP;
                        break;
                    }
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep > 0) tbest = std::min(tbest, ms);
                }
                if (status != SVR_OK) break;
                tbest += bin_ms;
                if (times_ms && nt < max_times) times_ms[nt] = tbest;
                ++nt;
                if (tbest < best) {
                    best = tbest;
                    best_cfg = c->cfg;
                }
            }
            if (status != SVR_OK) break;
        }
        if (status != SVR_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    release(pred);
    release(grads);
    if (status != SVR_OK) return status;
    rc = svr_set_config(c, &best_cfg);
    if (rc != SVR_OK) return rc;
    if (!c->binned) {
        rc = project_bin_impl(c, params);
        if (rc != SVR_OK) return rc;
    }
    c->tune_cache[key] = best_cfg;
    tune_cache_save(c, cache_path);
    *out = c->cfg;
    return SVR_OK;
}

}  // extern "C"
