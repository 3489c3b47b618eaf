// Internal definitions shared by the libsvr HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SVR_LOG2E 1.4426950408889634f
#define SVR_LN2 0.6931471805599453f
// exp(-x/2) = exp2(KZ * x)
#define SVR_KZ (-0.5f * SVR_LOG2E)

// Instance sort key = (global tile id << kClassBits) | footprint shape class.
// The binning sorts the tile bits only (a tile's instances stay in emission
// order); the tile kernels order a tile's instances by class in LDS.
constexpr int kClassBits = 6;
constexpr int kClasses = 1 << kClassBits;

// Static per-slice geometry (depends on the tile size through the tile table).
struct SliceGeo {
    float R0[9];
    float t0[3];
    float sig2[3];   // PSF variances along slice x, y, normal
    float dx, dy;
    int32_t H, W;
    int32_t ntx, nty;
    int32_t tile_base;  // first global tile id of the slice
    int32_t subject;
    int64_t pix_off;
};

// Per-iteration slice pose: R = Exp(omega) R0, t = t0 + tau.
struct SlicePose {
    float R[9];
    float t[3];
    float w[3];  // the rotation vector omega the frame was built from
    float pad;
};

// Per-iteration plane-test coefficients of a slice (built with its pose):
// unit normal n = R e_z, offset d = n . t, the products of n's components
// (n0^2, n1^2, n2^2, 2 n0 n1, 2 n0 n2, 2 n1 n2) and the through-plane PSF
// variance, so that m_z = n . mu - d and S'_zz = n^T Sigma n + sig2z cost
// three and six multiply-adds per (slice, Gaussian) candidate.
struct SlicePlane {
    float n[3];
    float d;
    float q[6];
    float sig2z;
    float pad;
};

struct SubjectInfo {
    int64_t g_begin, g_end;
    int32_t s_begin, s_end;
    // projection adjoint's per-slice pose sums: the subject's workgroups
    // (parts) are part0 .. part0 + nparts - 1; part k writes its 6 ns sums
    // at pose_base + k 6 ns, and the first reduction level writes nrc rows
    // of 6 ns (one per kPoseRowChunk parts) at pp_base
    int32_t part0, nparts, nrc, pad;
    int64_t pose_base, pp_base;
};
// workgroups of the projection adjoint per Gaussian block (256 Gaussians)
constexpr int kProjParts = 2;
constexpr int kPoseRowChunk = 64;  // parts per first-level row of the pose reduction

// Block table of the per-Gaussian kernels: blocks never straddle subjects.
struct GaussBlock {
    int64_t g_begin, g_end;
    int32_t subject;
    int32_t pad;
};

// Per-slice constants of the content-adaptive initialisation: reciprocals of
// the difference steps (1/(2 dx), 1/dx, 1/(2 dy), 1/dy, rounded once in FP64
// on the host) and the through-plane PSF FWHM (the slab of the jitter).
struct InitSlice {
    double inv2_x, inv1_x, inv2_y, inv1_y;
    float thick;
    int32_t pad;
};

// Normalised Top-K model (Eqs. 2 and 5): activated Gaussian, 48 B:
//   a = (mu, c), b = (S00, S01, S02, S11), c = (S12, S22, 0, 0) of Sigma_j.
struct TopkGauss {
    float4 a, b, c;
};
// Slice constants of the Top-K model: pose, P = R Sigma_PSF R^T (00 01 02 11
// 12 22) and the intensity scalar.
struct TopkSlice {
    float R[9];
    float t[3];
    float P[6];
    float sigma;
    float pad[3];
};
// Uniform cell grid of one subject's means for the neighbour search; cell
// (cx, cy, cz) has global id base + (cz * dims[1] + cy) * dims[0] + cx.
struct TopkGrid {
    float origin[3];
    float inv_h;
    float h;
    float rho0;          // first search radius (mm)
    int32_t dims[3];
    int32_t pad;
    int64_t base;
};

// One record = one (slice, Gaussian) pair that survives culling, 32 bytes.
//   r0 = (p*_x, p*_y, beta', amp)   centre in slice pixel units, beta' = KZ beta
//   r1 = (A'_00, A'_01, A'_11, slice id bits)  conic in pixel units times KZ
// The exponent of a pixel at pixel coordinates p is
//   z = beta' + A'_00 dx^2 + 2 A'_01 dx dy + A'_11 dy^2,  d = p - p*,
// and its value amp * max(exp2(z) - e_T, 0).
struct Record {
    float4 r0;
    float4 r1;
};

// Per-instance gradient (sums over the instance's pixels), two float4 per
// instance at its emission slot:
//   (d amp, d beta', d p*_x, d p*_y | d A'_00, d A'_01, d A'_11, unused)
// A record's instances occupy the contiguous slots rec_inst[r] = (first, count).

// Conditions recorded on the device by the library's calls, read and cleared
// by svr_check_status.
constexpr unsigned int kStatusCapacity = 1u;   // a fixed-capacity binning did not fit
constexpr unsigned int kStatusNonfinite = 2u;  // a finite check failed
struct DevStatus {
    unsigned int bits;
    int overflow;          // the last fixed-capacity binning did not fit (its binning is empty)
    long long need_rec;    // counts that binning needed
    long long need_inst;
};

// ---------------------------------------------------------------------------
// Host-side launchers (one per translation unit), all asynchronous on stream.
// ---------------------------------------------------------------------------
namespace svr {

// csrc/status.hip: any element of x [n] non-finite -> st->bits |= kStatusNonfinite.
hipError_t launch_check_finite(const float* x, int64_t n, DevStatus* st, hipStream_t s);
// Fixed-capacity binning: when totals [2] (records, instances) exceed the
// capacity, zero every Gaussian's counts and offsets [n] and record the
// needed counts.
hipError_t launch_fixed_capacity(const long long* totals, int64_t cap_rec, int64_t cap_inst, int2* counts,
                                 int2* offsets, int64_t n, DevStatus* st, hipStream_t s);
// Padding keys for instance slots [valid, cap), valid = 0 after an overflow
// else totals[1].
hipError_t launch_pad_instances(uint32_t* keys, uint32_t* vals, int64_t cap, const long long* totals,
                                const DevStatus* st, hipStream_t s);

struct ProjectArgs {
    const float* mean;
    const float* log_scale;
    const float* quat;
    const float* amp;
    const SliceGeo* geo;
    const SlicePose* pose;
    const SlicePlane* plane;  // per slice, with pose
    const SubjectInfo* subj;
    const GaussBlock* blocks;
    int32_t n_blocks;
    int32_t tile;
    float tau;
    // plane-test survivors from the count pass: bit (i - first slice of the
    // subject) of word [j * smask_words + (i - first) / 32] for Gaussian j
    uint32_t* smask;
    int32_t smask_words;
};

// plane (may be NULL): the slices' plane-test coefficients
hipError_t launch_slice_pose(const SliceGeo* geo, const float* pose, SlicePose* out, int32_t m,
                             hipStream_t st, SlicePlane* plane = nullptr);
hipError_t launch_cull_count(const ProjectArgs& a, int2* counts, hipStream_t st);
// fallback: int per Gaussian block (scratch, written by the first kernel)
// overflow (may be NULL): when *overflow != 0 the emission writes nothing.
hipError_t launch_emit(const ProjectArgs& a, const int2* counts, const int2* offsets, Record* rec,
                       int2* rec_inst, uint32_t* keys, uint32_t* vals, int* fallback, const int* overflow,
                       hipStream_t st);
// pose_part / pose_pp / w1: the two-level pose reduction (SubjectInfo); when
// max_subject_slices <= 512 the pose sums are reduced through them in a
// fixed order, else they are added to pose_acc atomically per record
hipError_t launch_project_backward(const ProjectArgs& a, const int2* offsets, const int2* counts,
                                   const Record* rec, const int2* rec_inst, const float4* inst_grad,
                                   int64_t n_inst, float* g_mean, float* g_log_scale, float* g_quat,
                                   float* g_amp, float* pose_acc, int32_t max_subject_slices, float* pose_part,
                                   float* pose_pp, const int4* w1, int32_t n_w1, const int2* w2, int32_t n_w2,
                                   int32_t m, hipStream_t st);
hipError_t launch_pose_chain(const float* pose, const float* pose_acc, float* g_pose, int32_t m,
                             hipStream_t st);

// Exclusive scan of int2 counts (component-wise) -> offsets, plus totals
// (int64 pair) written to totals[0..1].  tmp must hold scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
hipError_t launch_scan_int(const int* in, int* out, int64_t n, long long* totals, void* tmp, hipStream_t st);
hipError_t launch_scan_int2(const int2* in, int2* out, int64_t n, long long* totals, void* tmp,
                            hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on bits [first_bit, key_bits)
// of the key (the other bits are ignored and travel with the key).
// Buffers are ping-ponged; *result_in_alt tells where the result ended.  When
// idx/idx_alt are given, the input position of every pair travels with it
// (ending in the same buffer parity as keys).
size_t sort_tmp_bytes(int64_t n);
// Digit width (8 or 9 bits) the sort uses for a key of key_bits bits.
int radix_digit_bits(int key_bits);
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, int64_t n, int key_bits, void* tmp,
                             bool* result_in_alt, hipStream_t st, uint32_t* idx = nullptr,
                             uint32_t* idx_alt = nullptr, int first_bit = 0);

struct RenderArgs {
    const SliceGeo* geo;
    const int32_t* tile_slice;   // [n_tiles]
    const int4* tile_org;        // [n_tiles] origin of the tile (TileOrg packing)
    const int2* ranges;          // [n_tiles] [start, end) into sorted instances
    const uint32_t* inst_rec;    // sorted instance -> record id
    const uint32_t* inst_idx;    // sorted instance -> emission slot
    const uint32_t* inst_key;    // sorted instance -> key (tile << kClassBits | class)
    int64_t n_inst;              // sorted instances (emission padding included)
    const Record* rec;
    const int32_t* tile_order;   // persistent mode: tiles by decreasing cost (or NULL)
    int32_t n_tiles;
    int32_t tile;
    int32_t batch;
    int32_t persistent;
    int32_t forward_mode;        // 0: pixel per lane, 1: record per lane, 2: record on lanes
    int32_t loss_kind;           // 0: masked mean squared error, 1: masked L1 sum
    float etau;                  // exp(-T^2/2)
    float tau2;                  // T^2
    int32_t n_cu;                // compute units (persistent grid size)
};

// keys >= n_tiles (emission padding) are in no range; they are copied to
// pad_out (if not NULL) at their positions.
hipError_t launch_tile_ranges(const uint32_t* keys, int64_t n, int2* ranges, int32_t n_tiles,
                              uint32_t* pad_out, hipStream_t st);
hipError_t launch_mask_sum(const float* mask, int64_t n, float* partial, float* out,
                           hipStream_t st);
// partial: forward_partial_floats(a) floats of scratch (chunked record-per-lane mode).
hipError_t launch_forward(const RenderArgs& a, const float* target, const float* mask,
                          const float* msum, float* pred, float* grad_pred, float* tile_sse,
                          unsigned long long* incut, int* work_counter, float* partial, hipStream_t st);
size_t forward_partial_floats(const RenderArgs& a);
// Stable order of each tile's instances by shape class (keys, values and
// emission slots from the tile sort -> the _out arrays; ranges unchanged).
hipError_t launch_class_order(const uint32_t* keys, const uint32_t* vals, const uint32_t* idx, const int2* ranges,
                              int32_t n_tiles, uint32_t* keys_out, uint32_t* vals_out, uint32_t* idx_out,
                              hipStream_t st);
// Scale regulariser (adds to g [n,3] and, if loss != NULL, to loss[0]);
// partial holds kRegBlocks floats.
constexpr int kRegBlocks = 512;
hipError_t launch_scale_reg(const float* log_scale, int64_t n, float lambda, float s_target, float* g, float* loss,
                            float* partial, hipStream_t st);
hipError_t launch_loss_finalize(const float* tile_sse, const SliceGeo* geo, int32_t m,
                                const float* msum, float* slice_sse, float* loss, hipStream_t st);
hipError_t launch_backward(const RenderArgs& a, const float* grad_pred, const float* grad_scale,
                           float4* inst_grad, int* work_counter, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

struct AdamSeg {
    float* p;
    const float* g;
    int64_t n;
    int64_t state_off;
    float lr_a, lr_b;     // lr for the element (pose: a for omega, b for tau)
    int32_t pose_layout;  // 1: element e uses lr_a if e % 6 < 3 else lr_b
};
hipError_t launch_adam(const AdamSeg* segs, int n_segs, float* m, float* v, double beta1,
                       double beta2, double eps, double wd, int64_t step, hipStream_t st);

// Content-adaptive initialisation (Eq. 6).  sub_pix [s_n+1]: first pixel of
// each subject (sub_pix[s_n] = P).  launch_init_cdf writes the per-subject
// inclusive cumulative weights to cdf [P] and each subject's total weight to
// total [s_n]; scratch: g [P], gmax_bits [s_n], bsum [init_scan_blocks(P)],
// base [s_n].
int64_t init_scan_blocks(int64_t P);
hipError_t launch_init_cdf(const SliceGeo* geo, const InitSlice* tab, int32_t m, int32_t max_hw,
                           const int64_t* sub_pix, int32_t s_n, int64_t P, const float* image, const float* mask,
                           float lambda, double* g, unsigned long long* gmax_bits, int64_t* cdf, int64_t* bsum,
                           int64_t* base, int64_t* total, hipStream_t st);
hipError_t launch_init_sample(const SliceGeo* geo, const SlicePose* pose, const InitSlice* tab,
                              const SubjectInfo* subj, int32_t s_n, const int64_t* sub_pix, const int64_t* cdf,
                              const int64_t* total, const float* image, const float* u, int64_t N, float* mean,
                              int64_t* pixel, float* value, hipStream_t st);

// Per-slice outlier terms (csrc/outlier.hip); scratch holds
// slice_loss_partial_floats(m, max_hw) floats; msum is the mask sum (MSE).
size_t slice_loss_partial_floats(int32_t m, int32_t max_hw, int32_t s_n);
hipError_t launch_slice_loss(const SliceGeo* geo, const SubjectInfo* subj, int32_t s_n, int32_t m, int32_t max_hw,
                             const float* pred, const float* target, const float* mask, const float* sigma,
                             const float* log_omega, const float* msum, int32_t kind, float* loss, float* grad,
                             float* slice_sums, float* g_sigma, float* g_rho, float* scratch, hipStream_t st);

// Multiplicative bias field per subject (csrc/bias.hip): K <= kBiasMaxK basis
// Gaussians per subject, centres [S, K, 3], coefficients [S, K].
constexpr int kBiasMaxK = 64;
size_t bias_scratch_floats(int32_t m, int32_t max_hw, int32_t K);
hipError_t launch_bias_apply(const SliceGeo* geo, const SlicePose* pose, int32_t m, int32_t max_hw,
                             const float* centres, float width, const float* beta, int32_t K, float* pred,
                             float* bias, hipStream_t st);
// grad: dL/dy' in, dL/dy out; g_beta [S, K] overwritten; g_pose [M, 6] added to
hipError_t launch_bias_backward(const SliceGeo* geo, const SlicePose* pose, const SubjectInfo* subj, int32_t s_n,
                                int32_t m, int32_t max_hw, const float* centres, float width, const float* beta,
                                int32_t K, const float* pred_biased, const float* bias, float* grad,
                                float* g_beta, float* g_pose, float* scratch, hipStream_t st);

// Adaptive densification (csrc/densify.hip).
struct DensifyArgs {
    const float *mean, *log_scale, *quat, *amp;      // [n] parents
    const int32_t *n_out, *pos;                       // outputs per parent and their exclusive scan
    int64_t n, n_new;
    float *o_mean, *o_log_scale, *o_quat, *o_amp;    // [n_new]
    int32_t* src;                                     // [n_new]: j (kept) or -(j + 1) (child of j); may be NULL
    const float *m1_in, *m2_in;                       // Adam moments [11 n (+ pose)] or NULL
    float *m1_out, *m2_out;                           // [11 n_new (+ pose)]
    float log_scale_thr, split_offset, clone_offset;
    float split_dlog, split_amp;                      // 1/2 log(1 - a^2), 1 / (2 sqrt(1 - a^2))
};
hipError_t launch_densify_accumulate(const float* g_mean, float* acc, int32_t* cnt, int64_t n, hipStream_t st);
// n_out [n], pos [n] (exclusive scan), total (2 long long), new_off [S + 1];
// scan_tmp: scan_tmp_bytes(n)
hipError_t launch_densify_plan(const float* acc, const int32_t* cnt, const float* amp, int64_t n, float grad_thr,
                               float prune_amp, const SubjectInfo* subj, int32_t S, int32_t* n_out, int32_t* pos,
                               long long* total, void* scan_tmp, int64_t* new_off, hipStream_t st);
hipError_t launch_densify_emit(const DensifyArgs& a, hipStream_t st);

// Normalised Top-K model (csrc/topk.hip).
// gauss[s] is Gaussian perm[s] (cell order of the neighbour grid; NULL =
// identity).
hipError_t launch_topk_prepare(const float* mean, const float* log_scale, const float* quat, const float* amp,
                               int64_t n, const uint32_t* perm, const SlicePose* pose, const SliceGeo* geo,
                               const float* sigma, int32_t m, TopkGauss* gauss, TopkSlice* slices, hipStream_t st);
// bb [6 * n_subjects] order-preserving float keys (min xyz, max xyz)
hipError_t launch_topk_bbox(const float* mean, const GaussBlock* blocks, int32_t nb, int32_t n_subjects,
                            uint32_t* bb, hipStream_t st);
float topk_order_float(uint32_t k);
// *perm: the Gaussians in cell order (one of the value buffers).
hipError_t launch_topk_cells(const float* mean, const GaussBlock* blocks, int32_t nb, const TopkGrid* grid,
                             int64_t n, int64_t n_cells, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, void* sort_tmp, int key_bits, int2* cells, float4* smean,
                             const uint32_t** perm, hipStream_t st);
// status [2] (zeroed by the caller): pixels without K neighbours, sub-tile
// splits; max_tiles = the largest topk_knn_tiles over the slices
int32_t topk_knn_tiles(int32_t H, int32_t W);
hipError_t launch_topk_knn(const SliceGeo* geo, const TopkSlice* slices, const TopkGrid* grid, const int2* cells,
                           const float4* smean, const float* mask, int32_t m, int32_t max_tiles, int32_t K,
                           int32_t* nbr, int* status, hipStream_t st);
// Internal lists lint [K, n_act] (entry t of active pixel a at t * n_act +
// a): the lists of the active pixels with every id replaced by its
// cell-order position (iperm [N] scratch).
hipError_t launch_topk_internal(const int32_t* nbr, const int32_t* act, int64_t n_act, int32_t K,
                                const uint32_t* perm, int64_t n_gauss, int32_t* iperm, int32_t* lint, hipStream_t st);
// Inverse lists: entries of lint sorted by position; granges [N] per
// position, *gpix the sorted entry indices.
hipError_t launch_topk_inverse(const int32_t* lint, int64_t n_pairs, int64_t n_gauss, int key_bits,
                               uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                               void* sort_tmp, int2* granges, const uint32_t** gpix, hipStream_t st);
// Pixels with a list (nbr[p*K] >= 0) in 8x8-patch order: positions of
// slice i start at qoff[i] (its pixels padded to whole patches, Q in all);
// flag, off [Q] (off = exclusive scan, scan_tmp: scan_tmp_bytes(Q)),
// active [P] (0/1 per pixel), act [n_act] the pixels, act_off [M+1] each
// slice's range, total [2] with total[0] = n_act.
hipError_t launch_topk_active(const int32_t* nbr, int32_t K, const SliceGeo* geo, const int64_t* qoff, int32_t m,
                              int64_t Q, int* flag, int* off, uint8_t* active, int32_t* act, int32_t* act_off,
                              long long* total, void* scan_tmp, hipStream_t st);
int32_t topk_blocks_x(int32_t max_hw);
size_t topk_loss_partial_floats(int32_t m, int32_t max_hw, int32_t max_act);
hipError_t launch_topk_forward(const SliceGeo* geo, const TopkSlice* slices, const TopkGauss* gauss,
                               const int32_t* nbr, const int32_t* act, const int32_t* act_off, const uint8_t* active,
                               int64_t n_act, int32_t K, float delta, int32_t loss_kind, int32_t m, int32_t max_hw, int32_t max_act,
                               const float* target, const float* mask, const float* msum, float* pred, float2* state,
                               float* grad, float* partial, float* loss, hipStream_t st);
size_t topk_pose_partial_floats(int32_t m, int32_t max_act);
hipError_t launch_topk_backward(const SliceGeo* geo, const TopkSlice* slices, const TopkGauss* gauss,
                                const int32_t* nbr, const int32_t* act, const int32_t* act_off, int64_t n_act,
                                int32_t K, int32_t m, int32_t max_act, const float* grad_pred, const float2* state, const int2* granges,
                                const uint32_t* gpix, const uint32_t* perm, const float* log_scale, const float* quat,
                                int64_t n_gauss, float* g_mean, float* g_ls, float* g_quat, float* g_amp,
                                float* partial, float* pose_acc, float* g_sigma, float4* pxw, float2* pyd,
                                hipStream_t st);

}  // namespace svr
