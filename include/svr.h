/* svr.h -- C ABI of libsvr, the MI355X (gfx950) hot path of Gaussian-primitive
 * slice-to-volume reconstruction.
 *
 * The model (paper Sec. 2.1 Eq. 1, Sec. 2.3 Eqs. 3-5).  The high-resolution
 * volume is a field of N anisotropic Gaussians (Sec. 2.2): mean mu_j, scale
 * s_j = exp(log_scale_j), rotation from the quaternion q_j = (w,x,y,z)
 * (normalised on use), Sigma_j = R_j diag(s_j^2) R_j^T, amplitude c_j.  Slice i
 * has a nominal rotation R0_i (columns: slice x axis, slice y axis, normal) and
 * centre t0_i, a rigid 6-DoF pose delta (omega_i [rad], tau_i [mm]) with
 * R_i = Exp(omega_i) R0_i and t_i = t0_i + tau_i, pixel spacing (dx, dy), and a
 * Gaussian PSF with per-axis FWHM f (sigma = f / 2.355) in the slice frame.
 * Pixel (row r, column k) sits at u = ((k-(W-1)/2) dx, (r-(H-1)/2) dy, 0) in the
 * slice frame and at x = R_i u + t_i in the world.  The predicted pixel is
 *
 *   y = sum_j c_j sqrt(det Sigma_j / det Sigma_obs) max(exp(-q/2) - exp(-T^2/2), 0),
 *   Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T  (Eq. 4),  q = d^T Sigma_obs^-1 d,
 *   d = x - mu_j,
 *
 * over the Gaussians of the slice's subject, where T is the footprint cutoff
 * in standard deviations (3 by default): pairs beyond the T-sigma footprint
 * contribute nothing and the window is continuous at the cut.  The fitting
 * loss is the masked mean squared error L = sum m (y - I)^2 / sum m.
 *
 * Conventions for every call:
 *   - Every call returns an svr_status; nothing throws across the ABI.  On an
 *     error svr_last_error(ctx) describes it; outputs are then unspecified.
 *   - Pointers documented as DEVICE are device memory on the context's GPU,
 *     float32 (or the stated integer type), contiguous, 4-byte aligned, owned
 *     by the caller and never freed by the library.  HOST pointers are read
 *     during the call only.
 *   - All device work is enqueued asynchronously on the context's stream.
 *     svr_project_bin is the one call of the iteration that synchronises that
 *     stream (it reads the record and instance counts back), unless the
 *     context has a fixed capacity (svr_set_capacity); svr_get_stats with
 *     SVR_STATS_SYNC and svr_check_status also do.
 *   - Argument checks run on the host before any launch.
 *   - A context is not thread safe; use one context per host thread.
 */
#ifndef SVR_H
#define SVR_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define SVR_ABI_VERSION 2

typedef enum {
    SVR_OK = 0,
    SVR_ERR_ARG = -1,       /* invalid argument (null, size, range) */
    SVR_ERR_HIP = -2,       /* HIP runtime error or no usable GPU */
    SVR_ERR_CAPACITY = -3,  /* a count exceeds a representable or configured limit */
    SVR_ERR_STATE = -4,     /* calls out of order (e.g. forward before project_bin) */
    SVR_ERR_NODEVICE = -5,  /* compute call on a host-only context */
    SVR_ERR_NONFINITE = -6  /* a checked input or output is NaN or infinite (svr_set_checks) */
} svr_status;

typedef struct svr_ctx svr_ctx;

/* Library ABI version (SVR_ABI_VERSION). */
int svr_abi_version(void);

/* Human-readable name of a status code; never NULL. */
const char* svr_status_string(int status);

/* Create a context on GPU `device` that enqueues work on `hip_stream` (a
 * hipStream_t; NULL = the legacy default stream).  device = -1 creates a
 * host-only context that validates arguments and geometry but makes no HIP
 * call (compute calls then return SVR_ERR_NODEVICE).  Returns SVR_ERR_HIP if
 * the device cannot be used.  *out is NULL on failure. */
int svr_ctx_create(svr_ctx** out, int device, void* hip_stream);

/* Free the context and all device scratch it owns.  NULL is accepted. */
int svr_ctx_destroy(svr_ctx* ctx);

/* Change the stream subsequent calls enqueue on. */
int svr_set_stream(svr_ctx* ctx, void* hip_stream);

/* Message of the last failing call on this context ("" if none). */
const char* svr_last_error(const svr_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Acquisition geometry (Sec. 2.1, 2.3).  HOST arrays, copied into the
 * context; fixed until the next svr_set_geometry.  Subjects are independent
 * reconstructions batched together: subject s owns Gaussians
 * [gauss_offsets[s], gauss_offsets[s+1]) and the slices with slice_subject
 * == s, which must be contiguous and in nondecreasing subject order.  Pixels
 * of slice i are row-major and follow slice i-1 directly; the pixel offset of
 * slice i is sum_{k<i} height[k]*width[k].
 * Errors: SVR_ERR_ARG for null arrays, nonpositive sizes, unsorted subjects,
 * negative spacing/FWHM, non-monotone Gaussian offsets; SVR_ERR_CAPACITY when
 * the total pixel or tile count exceeds 2^31-1, a slice side exceeds 65535
 * pixels or a subject has more than 4096 slices. */
typedef struct {
    int32_t n_subjects;
    const int64_t* gauss_offsets;  /* [n_subjects+1], gauss_offsets[0] = 0 */
    int32_t n_slices;
    const int32_t* slice_subject;  /* [M] */
    const int32_t* height;         /* [M] rows, >= 1 */
    const int32_t* width;          /* [M] columns, >= 1 */
    const float* spacing;          /* [M,2] dx (between columns), dy (between rows), mm, > 0 */
    const float* psf_fwhm;         /* [M,3] slice-frame FWHM, mm, >= 0 */
    const float* rot0;             /* [M,9] row-major nominal rotation */
    const float* trans0;           /* [M,3] nominal slice centre, mm */
} svr_geometry;

int svr_set_geometry(svr_ctx* ctx, const svr_geometry* geom);

/* Total pixel count P of the current geometry (0 if none). */
int64_t svr_num_pixels(const svr_ctx* ctx);

/* Kernel configuration of the tile stages.  tile: 8, 16 or 32 (pixels per
 * tile side); batch: Gaussian records staged in LDS per step of the
 * pixel-per-lane forward, 32..256 and a multiple of 32; persistent: 0 = the
 * record-per-lane forward (mode 1) and the adjoint take fixed chunks of 256
 * tile-ordered instances per workgroup, modes 0 and 2 one workgroup per tile;
 * 1 = a persistent grid that pulls whole tiles from a work queue ordered by
 * decreasing instance count (every forward mode and the adjoint).  Chunks
 * suit workloads whose instances sit in few tiles, the work queue workloads
 * with many heavy tiles; svr_autotune measures both.  cutoff:
 * footprint radius T in
 * standard deviations, (0, 8]; forward_mode: 0 = pixel per lane (records
 * staged in LDS batches, deterministic summation order), 1 = record per lane
 * (each lane walks one record's footprint box and adds fixed-point terms to
 * an LDS pixel tile with integer atomics: exact per round of 256 records,
 * deterministic), 2 = record
 * on lanes (16-lane groups spread one record's footprint box over their
 * lanes and accumulate into their own LDS copy of the tile; deterministic).
 * Default {16, 128, 0, 3.0, 1}.  Changing tile or cutoff invalidates the last
 * svr_project_bin. */
typedef struct {
    int32_t tile;
    int32_t batch;
    int32_t persistent;
    float cutoff;
    int32_t forward_mode;
} svr_config;

int svr_set_config(svr_ctx* ctx, const svr_config* cfg);

/* Data term of the objective, used by svr_forward's loss outputs (default
 * SVR_LOSS_MSE):
 *   SVR_LOSS_MSE  masked mean squared error L = sum m (y - I)^2 / sum m,
 *                 grad_pred = 2 m (y - I) / sum m, slice_sse = per-slice
 *                 sums of m (y - I)^2;
 *   SVR_LOSS_L1   the paper's L1 data term (Sec. 2.5, Eq. 7) with the mask,
 *                 L = sum m |y - I| (not normalised), grad_pred =
 *                 m sign(y - I) (0 where y = I), slice_sse = per-slice sums
 *                 of m |y - I|.
 * Errors: SVR_ERR_ARG for an unknown kind. */
#define SVR_LOSS_MSE 0
#define SVR_LOSS_L1 1
int svr_set_loss(svr_ctx* ctx, int kind);

/* Scale regulariser of Eq. 7 (Sec. 2.5): for the n Gaussians' scales
 * s = exp(log_scale) [n,3] (DEVICE), adds lambda sum_j ||s_j - s_target||^2
 * to loss[0] (DEVICE, may be NULL) and 2 lambda (s - s_target) s to
 * g_log_scale [n,3] (DEVICE), both in place, on the context's stream.  Call it
 * after svr_backward, which overwrites the gradients.  The paper uses
 * lambda = 2.5e-3 and s_target = 1.6 mm with its L1 term.  Errors:
 * SVR_ERR_ARG for n < 0, NULL arrays with n > 0, lambda < 0 or not finite,
 * s_target <= 0 or not finite. */
int svr_scale_regularizer(svr_ctx* ctx, const float* log_scale, int64_t n, float lambda, float s_target,
                          float* g_log_scale, float* loss);
int svr_get_config(const svr_ctx* ctx, svr_config* cfg);

/* ------------------------------------------------------------------------ */
/* Content-adaptive initialisation of the means (Sec. 2.5, Eq. 6).  Each
 * pixel of the current geometry gets the weight
 *   w = floor(2^20 ((1 - lambda_init) ||grad I|| / gmax + lambda_init))
 * if mask > 0 (0 otherwise), where ||grad I|| is the in-slice gradient
 * magnitude of image in intensity per mm (central differences inside the
 * slice, one-sided on its border, 0 along an axis of length 1) and gmax its
 * largest value over the subject's masked pixels (if gmax = 0 the weight is
 * floor(2^20 lambda_init)).  The weights are computed in FP64 with each
 * operation rounded once, so they are exact integers that any conforming
 * implementation reproduces.
 *
 * svr_init_cdf writes the inclusive cumulative weights, restarting at each
 * subject's first pixel, to cdf [P] (DEVICE int64), and each subject's total
 * weight to totals [n_subjects] (HOST, may be NULL).  Synchronous.
 *
 * svr_init_means draws a pixel for every Gaussian j of subject s from its
 * subject's weights: with W the subject's total and u = u[j] [N,4] (DEVICE,
 * uniforms in [0, 1), 16-byte aligned), t = min(floor(u.x W), W - 1) and the
 * pixel is the first whose cumulative weight exceeds t; the mean is the
 * pixel centre moved by ((u.y - 1/2) dx, (u.z - 1/2) dy, (u.w - 1/2) FWHM_z)
 * in the slice frame, mapped to the world by the slice pose pose [M,6]
 * (DEVICE, as in svr_params).  Writes mean [N,3] (DEVICE), and if not NULL
 * pixel [N] (DEVICE int64, global pixel index) and value [N] (DEVICE, image
 * at that pixel).  Synchronous up to the final sampling launch, which is
 * asynchronous on the context's stream; uses about 16 B of device scratch
 * per pixel, kept until the context is destroyed.
 *
 * image [P] and mask [P] (DEVICE, mask may be NULL = all pixels) must be
 * finite.  Errors: SVR_ERR_STATE without geometry; SVR_ERR_ARG for NULL
 * image / cdf / pose / u / mean, lambda_init outside [0, 1], a misaligned u,
 * or a subject with Gaussians whose weights are all 0 (every pixel masked
 * out, or lambda_init = 0 on a constant image). */
int svr_init_cdf(svr_ctx* ctx, const float* image, const float* mask, float lambda_init, int64_t* cdf,
                 int64_t* totals);
int svr_init_means(svr_ctx* ctx, const float* image, const float* mask, const float* pose, float lambda_init,
                   const float* u, float* mean, int64_t* pixel, float* value);

/* ------------------------------------------------------------------------ */
/* Parameters: DEVICE pointers, float32.
 *   mean [N,3], log_scale [N,3], quat [N,4] (w,x,y,z, nonzero), amp [N],
 *   pose [M,6] = (omega_x, omega_y, omega_z [rad], tau_x, tau_y, tau_z [mm]). */
typedef struct {
    const float* mean;
    const float* log_scale;
    const float* quat;
    const float* amp;
    const float* pose;
} svr_params;

/* Gradients: DEVICE pointers with the shapes of svr_params, overwritten. */
typedef struct {
    float* mean;
    float* log_scale;
    float* quat;
    float* amp;
    float* pose;
} svr_grads;

/* Cull, project and bin (Sec. 2.3 Eq. 4 evaluated per slice and Gaussian;
 * replaces the paper's Top-K neighbour search of Sec. 2.5).
 * For every slice i and Gaussian j of the same subject, keeps the pair when
 * the slice plane crosses j's T-sigma footprint (minimum of q over the plane
 * <= T^2), writes one record (in-plane centre, in-plane conic, amplitude,
 * through-plane term) and one instance per overlapped pixel tile, then sorts
 * the instances by (slice, tile) with a stable LDS radix sort and builds
 * per-tile ranges.  The records stay valid until the next call; svr_forward
 * and svr_backward use them and assume the parameters have not changed.
 * Synchronises the stream once to read the counts (not in fixed-capacity
 * mode, see svr_set_capacity).  Errors: SVR_ERR_STATE without geometry,
 * SVR_ERR_ARG for null pointers or N different from the geometry's Gaussian
 * count, SVR_ERR_CAPACITY above 2^31-1 records or instances,
 * SVR_ERR_NONFINITE (with SVR_CHECK_FINITE) for a non-finite parameter. */
int svr_project_bin(svr_ctx* ctx, const svr_params* params);

/* Forward model and masked-MSE loss (Eq. 5 with the exact amplitude; the
 * masked MSE replaces Eq. 7's L1 term).  pred [P] DEVICE is overwritten with
 * the predicted pixels.  When target [P] and mask [P] (DEVICE, mask in {0,1})
 * are given, the optional outputs are written: loss [1] = sum m (y-I)^2 /
 * sum m, slice_sse [M] = per-slice sum m (y-I)^2, grad_pred [P] = dL/dy =
 * 2 m (y - I) / sum m.  Any of them may be NULL.  A mask summing to zero
 * gives loss 0 and grad 0.  Errors: SVR_ERR_STATE before svr_project_bin,
 * SVR_ERR_ARG for a requested output without target and mask. */
int svr_forward(svr_ctx* ctx, const float* target, const float* mask, float* pred,
                float* loss, float* slice_sse, float* grad_pred);

/* Adjoint of svr_forward: with g = grad_pred [P] (DEVICE) scaled by
 * *grad_scale (DEVICE float [1], NULL = 1), writes the gradient of
 * sum_p g_p y_p with respect to every parameter of the last svr_project_bin
 * (Gaussian mean, log_scale, quaternion, amplitude and slice poses; the pose
 * gradient is with respect to (omega, tau) through the left Jacobian of
 * SO(3)).  Pixel-Gaussian terms are recomputed per tile, no per-pair state is
 * kept.  Errors: SVR_ERR_STATE before svr_project_bin, SVR_ERR_ARG for null
 * pointers. */
int svr_backward(svr_ctx* ctx, const float* grad_pred, const float* grad_scale,
                 const svr_grads* out);

/* ------------------------------------------------------------------------ */
/* The paper's normalised Top-K forward model (Eqs. 2 and 5 with the Top-K
 * neighbour sets of Sec. 2.5), as an alternative to the windowed model of
 * svr_project_bin / svr_forward.  For pixel p of slice i at
 * x = R_i u_p + t_i:
 *   y_p = sigma_i N_p / (D_p + delta),  N_p = sum_j c_j e_j,  D_p = sum_j e_j,
 *   e_j = exp(-1/2 v^T Sigma_obs^-1 v),  v = x - mu_j,
 *   Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T,
 * the sums over the K means of the slice's subject nearest to x (L2), as in
 * Eq. 5 without the sqrt(det) factor of the windowed model.
 *
 * svr_topk_build computes those neighbour lists for the current geometry
 * from mean [N,3] and pose [M,6] (DEVICE) for every pixel with mask > 0
 * (mask [P] DEVICE, NULL = every pixel) and writes them to nbr [P,K]
 * (DEVICE int32, caller-owned, global Gaussian ids in no particular order;
 * a pixel outside the mask gets -1 in every entry and is predicted as 0, so
 * pass the same mask to the forward).
 * The paper refreshes its neighbour index every 50 epochs: the lists are
 * then reused with changing parameters until the next build.  The context
 * also keeps the inverse lists (the pixels holding each Gaussian, 8 B per
 * list entry plus sort space, about 4 x 4 B x P x K in total) for the
 * adjoint.  Synchronous.  Errors: SVR_ERR_STATE without geometry;
 * SVR_ERR_ARG for NULL pointers, K outside [1, 1024] or a subject with
 * slices and fewer than K Gaussians; SVR_ERR_CAPACITY when P*K exceeds
 * 2^31-1 or the search cannot complete for some pixel (more than 2,560
 * means within reach of one pixel, or fewer than K within about 60 times
 * the mean neighbour distance).
 *
 * svr_topk_forward evaluates the model with params (svr_params), sigma [M]
 * (DEVICE, per-slice intensity scalars of Sec. 2.4, NULL = all 1), delta > 0
 * and the nbr / K of the last build, writing pred [P].  With target and
 * mask (DEVICE [P]) it also writes the loss of the context's loss kind
 * (svr_set_loss: masked MSE or L1) to loss [1] and dL/dy to grad_pred [P];
 * either may be NULL.  It keeps N_p / (D_p + delta) and D_p + delta per pixel
 * for the adjoint.
 *
 * svr_topk_backward writes the gradient of sum_p g_p y_p, g = grad_pred [P]
 * (DEVICE), with respect to the parameters of the last svr_topk_forward
 * (mean, log_scale, quat, amp, and pose through the left Jacobian of SO(3))
 * to out, and with respect to sigma to g_sigma [M] (DEVICE, may be NULL).
 * Pixels with g_p = 0 are skipped.  The lists are held fixed (the gradient
 * of the selection itself is zero almost everywhere).  Errors: SVR_ERR_STATE
 * before a build or forward, or for nbr / K other than the build's;
 * SVR_ERR_ARG for NULL pointers or delta <= 0. */
int svr_topk_build(svr_ctx* ctx, const float* mean, const float* pose, const float* mask, int K, int32_t* nbr);
int svr_topk_forward(svr_ctx* ctx, const svr_params* params, const float* sigma, const int32_t* nbr, int K,
                     float delta, const float* target, const float* mask, float* pred, float* loss,
                     float* grad_pred);
int svr_topk_backward(svr_ctx* ctx, const svr_params* params, const int32_t* nbr, int K, const float* grad_pred,
                      const svr_grads* out, float* g_sigma);

/* ------------------------------------------------------------------------ */
/* Per-slice outlier terms (Sec. 2.4) on a prediction pred [P] (DEVICE) from
 * svr_forward or svr_topk_forward called without target: the learnable
 * intensity scalar sigma_i (the slice is predicted as sigma_i y) and the
 * aleatoric weight omega_i = exp(rho_i) that down-weights a slice.  The
 * paper gives no loss form for omega_i; it is read as a per-slice
 * likelihood scale, with r = sigma_i y - I, S_i the slice's masked data sum
 * and n_i its mask sum:
 *   SVR_LOSS_MSE:  L = (sum_i e^{-2 rho_i} S_i + 2 n_i rho_i) / sum m,
 *                  S_i = sum m r^2  (Gaussian, standard deviation omega_i);
 *   SVR_LOSS_L1:   L = sum_i e^{-rho_i} S_i + n_i rho_i,
 *                  S_i = sum m |r|  (Laplace, scale omega_i);
 * both equal the plain data terms at sigma = 1, rho = 0.  A common factor on
 * a subject's sigma_i trades against its amplitudes, and a common shift of
 * its rho_i rescales its data term against any regulariser; the terms above
 * therefore use the per-subject centred sigma_i / geomean(sigma) and
 * rho_i - mean(rho), and the gradients with respect to log sigma and rho sum
 * to zero over each subject.  Inputs: target,
 * mask [P], sigma [M] and log_omega [M] = rho (DEVICE; sigma / log_omega
 * NULL = 1 / 0).  Outputs (DEVICE, each may be NULL): loss [1], grad_pred
 * [P] = dL/dy (pass it to svr_backward / svr_topk_backward), slice_sums [M]
 * = S_i, g_sigma [M], g_log_omega [M].  Asynchronous.  Errors:
 * SVR_ERR_STATE without geometry, SVR_ERR_ARG for NULL pred / target /
 * mask. */
int svr_slice_loss(svr_ctx* ctx, const float* pred, const float* target, const float* mask, const float* sigma,
                   const float* log_omega, float* loss, float* grad_pred, float* slice_sums, float* g_sigma,
                   float* g_log_omega);

/* Multiplicative low-frequency bias field per subject, a reading of the
 * paper's bias-field Gaussians (Sec. 4, "Bias Correction & Robustness"; the
 * paper gives no form): subject s has K fixed broad basis Gaussians with
 * centres m_{s,k} and one width w, and coefficients beta_{s,k};
 *   b(x) = exp(sum_k beta_{s,k} exp(-|x - m_{s,k}|^2 / (2 w^2)))
 * at every pixel's world position x_p = R_i u_p + t_i under the poses of the
 * last svr_project_bin (the field moves with the subject; the context keeps
 * its own copy of the slice frames, so the caller's pose array may change
 * after that call).  beta = 0 gives
 * b = 1.
 *
 * svr_bias_apply: pred [P] <- b(x_p) pred[p] in place (call it after
 * svr_forward without target and before the loss, e.g. svr_slice_loss);
 * bias [P] (may be NULL) receives b.  centres [S*K*3], beta [S*K], pred and
 * bias are DEVICE pointers; 1 <= K <= SVR_BIAS_MAX_K, width > 0.
 * Asynchronous.  Errors: SVR_ERR_STATE before svr_project_bin, SVR_ERR_ARG
 * for NULL centres / beta / pred or K / width out of range. */
#define SVR_BIAS_MAX_K 64
int svr_bias_apply(svr_ctx* ctx, const float* centres, float width, const float* beta, int32_t K, float* pred,
                   float* bias);

/* Adjoint of svr_bias_apply for the loss L(y'), y' = b y: grad_pred [P]
 * holds dL/dy' on entry and dL/dy = b dL/dy' on return (pass it on to
 * svr_backward); g_beta [S*K] receives dL/dbeta = sum_p dL/dy'_p y'_p phi_k;
 * g_pose [M*6] (may be NULL) has the field's pose terms ADDED to it (through
 * x_p: dL/dtau = sum dL/dx_p, dL/domega = J_l(omega)^T sum (R_i u_p) x
 * dL/dx_p, the convention of svr_backward's pose gradient), so call it
 * after svr_backward when both are wanted.  pred_biased [P] = y' and bias
 * [P] = b from svr_bias_apply with the same arguments.  All DEVICE pointers.
 * Sums have a fixed order (deterministic).  Asynchronous.  Errors as
 * svr_bias_apply, plus SVR_ERR_ARG for NULL pred_biased / bias / grad_pred /
 * g_beta. */
int svr_bias_backward(svr_ctx* ctx, const float* centres, float width, const float* beta, int32_t K,
                      const float* pred_biased, const float* bias, float* grad_pred, float* g_beta, float* g_pose);

/* ------------------------------------------------------------------------ */
/* Adaptive densification, a reading of the paper's coarse-to-fine future
 * work (Sec. 4, "Coarse-to-Fine Optimization": progressive densification
 * after 3D Gaussian Splatting, starting from few large primitives); the
 * paper gives no rule, so the clone/split scheme of 3DGS is taken with its
 * statistic in this model's world frame.
 *
 * svr_densify_accumulate: after svr_backward, A_j += ||dL/dmu_j|| and
 * n_j += 1 where dL/dmu_j is not zero.  g_mean [N*3], grad_acc [N] (float),
 * count [N] (int32), all DEVICE; the caller zeroes A and n when it starts a
 * new statistic.  Asynchronous.  Errors: SVR_ERR_STATE without geometry,
 * SVR_ERR_ARG for NULL arrays. */
int svr_densify_accumulate(svr_ctx* ctx, const float* g_mean, float* grad_acc, int32_t* count);

typedef struct {
    float grad_threshold;       /* densify j when n_j > 0 and A_j > fl(grad_threshold * n_j) (FP32), >= 0 */
    float log_scale_threshold;  /* a densified j splits when max_k log s_jk > this, else it is cloned */
    float split_offset;         /* a in (0, 1): split children at mu -+ a s_a e, s_a *= sqrt(1 - a^2),
                                   c *= 1 / (2 sqrt(1 - a^2)); sqrt(3)/2 halves s_a and keeps c */
    float clone_offset;         /* b >= 0: clone children at mu -+ b s_a e, same shape, c / 2 */
    float prune_amp;            /* drop j when |c_j| < prune_amp (0: never); pruning wins over densifying */
} svr_densify_cfg;

/* svr_densify: the densified mixture of the current one.  e is the principal
 * axis of Sigma_j (the column of R(q_j) of the largest scale s_a, the first
 * on ties); a split keeps the parent's integral and first two moments, a
 * clone its integral and mean.  in: the current mean [N*3], log_scale
 * [N*3], quat [N*4], amp [N] (in->pose unused); grad_acc, count: the
 * statistic above.  out: mean, log_scale, quat, amp arrays with room for
 * `capacity` Gaussians (out->pose unused).  Outputs stay grouped by subject
 * and in parent order; a densified parent is replaced by its two children
 * ("-" first).  src [capacity] (may be NULL) receives j for a kept Gaussian
 * and -(j + 1) for a child of j.  exp_avg_in / exp_avg_sq_in [11 N + 6 M]
 * and exp_avg_out / exp_avg_sq_out [11 K + 6 M] (the svr_step layout; all
 * four or none; not in place): the moments of kept Gaussians are carried
 * over, children start from zero, the pose part is copied.  new_offsets
 * (HOST, [S + 1]) always receives the new per-subject Gaussian offsets; K =
 * new_offsets[S].  All other pointers are DEVICE.  Synchronous (the new
 * offsets are read back).  On success the context takes the new offsets
 * (as svr_set_geometry would with the same slices): the next
 * svr_project_bin expects the new arrays, and the binning and Top-K state
 * are invalidated.  Errors: SVR_ERR_CAPACITY when K > capacity (only
 * new_offsets is written, the context is unchanged) or 2 N > 2^31 - 1;
 * SVR_ERR_ARG for NULL arrays or out-of-range parameters; SVR_ERR_STATE
 * without geometry. */
int svr_densify(svr_ctx* ctx, const svr_params* in, const float* grad_acc, const int32_t* count,
                const svr_densify_cfg* cfg, const svr_grads* out, int64_t capacity, int32_t* src,
                const float* exp_avg_in, const float* exp_avg_sq_in, float* exp_avg_out, float* exp_avg_sq_out,
                int64_t* new_offsets);

/* AdamW (App. A.1).  lr[6] = learning rates of the groups mean, log_scale,
 * quat, amp, pose rotation omega, pose translation tau.  Updates params,
 * exp_avg and exp_avg_sq in place; step counts from 1 (bias correction).
 * exp_avg / exp_avg_sq are DEVICE float32 [N*11 + M*6], laid out as
 * mean (3N), log_scale (3N), quat (4N), amp (N), pose (6M).  Follows
 * torch.optim.AdamW: p *= 1 - lr*wd; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr/(1-b1^t) * m / (sqrt(v)/sqrt(1-b2^t) + eps).
 * Errors: SVR_ERR_ARG for null pointers, step < 1, betas outside [0,1). */
typedef struct {
    float lr[6];
    double beta1, beta2, eps, weight_decay;  /* double so that 1 - beta is exact on the host */
} svr_adam;

int svr_step(svr_ctx* ctx, const svr_grads* params_inout, const svr_grads* grads,
             float* exp_avg, float* exp_avg_sq, const svr_adam* hp, int64_t step);

/* The same AdamW update on one plain vector p [n] with gradient g [n] and
 * moments exp_avg / exp_avg_sq [n] (all DEVICE), learning rate lr (hp->lr is
 * not used): for per-slice parameters such as sigma and log_omega.
 * Errors: SVR_ERR_ARG for null pointers, n < 0, step < 1, bad betas. */
int svr_adam_vector(svr_ctx* ctx, float* p, const float* g, float* exp_avg, float* exp_avg_sq, int64_t n, float lr,
                    const svr_adam* hp, int64_t step);

/* Counters of the last svr_project_bin / svr_forward.  Record and instance
 * counts are exact after svr_project_bin (in fixed-capacity mode only after a
 * call with SVR_STATS_SYNC, which reads them from the device).
 * n_fallback_blocks is read (synchronising the stream) only with
 * SVR_STATS_SYNC.  n_incut (pairs inside the cutoff,
 * i.e. Gaussian-pixel terms that contribute) is counted by svr_forward only
 * when flags has SVR_STATS_SYNC set at the *next* svr_get_stats call after a
 * forward run with counting enabled via svr_set_count_pairs(ctx, 1); the
 * call then synchronises the stream. */
typedef struct {
    int64_t n_gauss;
    int64_t n_slices;
    int64_t n_pixels;
    int64_t n_tiles;
    int64_t n_candidates;   /* (slice, Gaussian) pairs tested */
    int64_t n_records;      /* pairs kept (plane crosses the footprint, bbox non-empty) */
    int64_t n_instances;    /* (tile, record) pairs */
    int64_t n_incut;        /* (pixel, Gaussian) pairs with q < T^2; -1 if not counted */
    int64_t n_evaluated;    /* pixel-record evaluations the forward tile kernel performs */
    int32_t key_bits;       /* bits of the sort key */
    int32_t sort_passes;
    int64_t n_fallback_blocks;  /* Gaussian blocks of 256 whose records exceeded the emission
                                   kernel's LDS list and were emitted per lane; -1 if not read */
} svr_stats;

#define SVR_STATS_SYNC 1
int svr_set_count_pairs(svr_ctx* ctx, int enable);
int svr_get_stats(svr_ctx* ctx, int flags, svr_stats* out);

/* ------------------------------------------------------------------------ */
/* Fixed-capacity binning (no host synchronisation).  By default
 * svr_project_bin reads the record and instance counts back to size its
 * buffers, which synchronises the stream once per call.  svr_set_capacity
 * with max_records > 0 and max_instances > 0 allocates the binning buffers
 * for those counts now (this call synchronises) and switches svr_project_bin
 * to a mode that never reads back, never allocates and never synchronises:
 * counts stay on the device, the sort and the tile stages always cover
 * max_instances slots (unused slots carry a padding key that sorts after every
 * tile and is skipped), so their cost follows the capacity, not the count.
 * When a call needs more records or instances than the capacity, it writes
 * nothing out of bounds: the binning is left empty (every prediction and
 * gradient of that iteration is 0) and the condition is recorded on the
 * device; svr_check_status then returns SVR_ERR_CAPACITY with the needed
 * counts.  max_records = max_instances = 0 returns to the default mode.
 * Errors: SVR_ERR_ARG for negative values or only one of them 0,
 * SVR_ERR_CAPACITY above 2^31-1, SVR_ERR_HIP if the allocation fails. */
int svr_set_capacity(svr_ctx* ctx, int64_t max_records, int64_t max_instances);

/* Finite checks.  With flags & SVR_CHECK_FINITE, svr_project_bin checks
 * every Gaussian parameter and slice pose, svr_forward every predicted
 * pixel and svr_backward every gradient it writes, on the device.  A
 * non-finite value is recorded on the device; svr_project_bin in the default
 * mode returns SVR_ERR_NONFINITE itself (it synchronises anyway, and then
 * leaves the binning invalid), the other calls report it through
 * svr_check_status.  Default: no checks (they cost one extra read of the
 * checked arrays).  Errors: SVR_ERR_ARG for unknown flags. */
#define SVR_CHECK_FINITE 1
int svr_set_checks(svr_ctx* ctx, int flags);

/* Synchronises the context's stream and returns the conditions recorded on
 * the device since the last svr_check_status (or project_bin that reported
 * one), then clears them: SVR_ERR_CAPACITY (a fixed-capacity binning was too
 * small; needed_records / needed_instances, HOST, may be NULL, receive the
 * counts it needed), else SVR_ERR_NONFINITE (a finite check failed), else
 * SVR_OK. */
int svr_check_status(svr_ctx* ctx, int64_t* needed_records, int64_t* needed_instances);

/* Stable radix sort used by tile binning, exposed for verification: sorts the
 * n (key, value) pairs in place by the low key_bits bits of the key (1..32),
 * keeping the input order of equal keys; bits above key_bits are ignored for
 * the order and kept in the output.  keys/vals are DEVICE uint32 [n];
 * scratch is owned by the context.  Errors: SVR_ERR_ARG for null pointers with n > 0,
 * n < 0 or key_bits outside 1..32. */
int svr_sort_pairs(svr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int key_bits);

/* Allocation-free variant of svr_sort_pairs, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and result as svr_sort_pairs (the
 * same kernels: bit-identical output), with these differences:
 *   - n <= SVR_SORT_NOALLOC_MAX, else SVR_ERR_CAPACITY (checked on the host);
 *   - nothing is allocated or freed and the stream is not synchronised: the
 *     sort is enqueued on the context's stream and has finished when that
 *     stream has;
 *   - its scratch (ping-pong keys and values and the pass histograms, 11 MiB)
 *     is one fixed device array per GPU, held from the library's first
 *     context on that GPU until the process ends.  Every call on a GPU uses
 *     that GPU's array, so calls that overlap on one GPU (several streams,
 *     contexts or host threads) race: the caller must order them.  Nothing in
 *     the array needs to start at zero.
 * Errors: as svr_sort_pairs; SVR_ERR_NODEVICE on a host-only context. */
#define SVR_SORT_NOALLOC_MAX (1 << 20)
int svr_sort_pairs_noalloc(svr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int key_bits);

/* Per-stage GPU timing.  When enabled, every stage the library launches is
 * bracketed by HIP events on the context stream; svr_get_timing synchronises
 * the stream, folds the completed intervals into per-stage totals and copies
 * up to max_out entries (HOST array) in a fixed stage order, setting *n_out.
 * Stage names: slice_pose, cull_count, scan, emit, sort, tile_ranges,
 * tile_order, mask_sum, forward_tile, loss_reduce, zero_fill, backward_tile,
 * project_backward, pose_chain, adam, topk_knn, topk_inverse, topk_forward,
 * topk_backward.  Enabling or disabling clears the totals.  An event record
 * can leave the GPU idle for several microseconds between kernels, so a
 * caller timing whole iterations should bracket only the stages it needs
 * (svr_set_timing_stages). */
typedef struct {
    char name[32];
    int64_t calls;
    double total_ms;
} svr_timer;

int svr_set_timing(svr_ctx* ctx, int enable);
int svr_get_timing(svr_ctx* ctx, svr_timer* out, int max_out, int* n_out);
/* Stages that timing brackets with events: bit s of mask selects stage s in
 * the order listed above (default: all).  Takes effect for stages launched
 * afterwards; totals are kept.  Errors: SVR_ERR_ARG for a null context. */
int svr_set_timing_stages(svr_ctx* ctx, uint32_t mask);

/* ------------------------------------------------------------------------ */
/* Autotuner (batched launch).  Times binning (svr_project_bin) and the
 * forward and backward passes for every tile size in {8,16,32}, forward mode in
 * {0,1,2}, LDS batch in {32,64,128,256} (mode 0) and persistent in {0,1}
 * (those allowed by flags), picks the
 * fastest and makes it the context's configuration (re-binning when the tile
 * size changes).  params/grad_pred as in svr_project_bin / svr_backward
 * (grad_pred may be any DEVICE buffer of P floats).  Results are cached in the
 * context per shape bucket (pixels and records rounded to powers of two, and
 * the subject count: none of them depends on the configuration) and, when
 * cache_path is non-NULL, in a small text file there.
 * out receives the chosen configuration; times_ms (HOST, may be NULL)
 * receives up to max_times measured (binning + forward + backward) times in
 * trial order.  Synchronises the stream. */
#define SVR_TUNE_TILE 1
#define SVR_TUNE_BATCH 2
#define SVR_TUNE_PERSISTENT 4
#define SVR_TUNE_MODE 8
#define SVR_TUNE_ALL 15
int svr_autotune(svr_ctx* ctx, const svr_params* params, const float* grad_pred, int flags,
                 const char* cache_path, svr_config* out, float* times_ms, int max_times);

/* ------------------------------------------------------------------------ */
/* Learned pose proposal.  A small CNN maps a 128x128 crop of an observed
 * slice (its 32x32 centre upsampled x4, bilinear) plus the slice's nominal
 * placement (stack rotation R0, 9 floats, and nominal centre t0 / 16 mm, 3
 * floats) to a 6-DoF pose delta (omega, tau) that initialises the
 * slice's pose; the plain pose optimisation has the last word (a proposal is
 * only kept where it lowers the slice's forward-model error).  Architecture:
 * 6 x [3x3 conv, stride 2, pad 1, ReLU] with 32, 32, 64, 64, 128, 128
 * channels (128^2 -> 2^2), flatten (512) || placement (12), FC 524 -> 256
 * (ReLU), FC 256 -> 6.  Every layer runs as an implicit GEMM on BF16 MFMA
 * with FP32 accumulation; master weights, activations and Adam state are
 * FP32.  Targets/outputs are in the caller's units (the training code uses
 * scaled pose units).  All array arguments are DEVICE float32 pointers in
 * NCHW / row-major layout, except the HOST arrays of get/set_params. */
typedef struct svr_posenet svr_posenet;

/* Create with He-normal weights from `seed` on GPU `device`, enqueueing on
 * `hip_stream`; max_batch bounds B in every call (1..65536). */
int svr_posenet_create(svr_posenet** out, int device, void* hip_stream, uint64_t seed, int max_batch);
int svr_posenet_destroy(svr_posenet* net);
int64_t svr_posenet_num_params(const svr_posenet* net);
/* Flat parameter vector: per conv layer weight [Co,Ci,3,3] then bias [Co];
 * fc1 weight [256,524], bias [256]; fc2 weight [6,256], bias [6]. */
int svr_posenet_get_params(svr_posenet* net, float* host_out);
int svr_posenet_set_params(svr_posenet* net, const float* host_in);
/* slices [B,H,W] -> crops [B,128,128]: the centred 32x32 window upsampled x4. */
int svr_posenet_prepare(svr_posenet* net, const float* slices, int B, int H, int W, float* crops);
/* crops [B,1,128,128], placement [B,12] -> out [B,6]. */
int svr_posenet_forward(svr_posenet* net, const float* crops, const float* orient, int B, float* out);
/* One Adam step (betas 0.9/0.999, eps 1e-8) on loss = mean_b sum_c (y-t)^2;
 * loss [1] (DEVICE, may be NULL) receives the batch loss before the step. */
int svr_posenet_train_step(svr_posenet* net, const float* crops, const float* orient, const float* target,
                           int B, float lr, float* loss);
/* Loss and the full parameter gradient (grads_out [num_params], DEVICE),
 * without updating the weights. */
int svr_posenet_grads(svr_posenet* net, const float* crops, const float* orient, const float* target, int B,
                      float* loss, float* grads_out);

/* Layer primitives of the network (on the given hipStream_t), exposed for
 * verification.  conv: x [B,Ci,H,W], w [Co,Ci,3,3], b [Co] (may be NULL),
 * y [B,Co,(H+1)/2,(W+1)/2]; relu = 1 applies max(.,0).  dgrad/wgrad take dy
 * (gradient w.r.t. y) and y (the ReLU output, NULL for no ReLU); dgrad writes
 * dx [B,Ci,H,W], wgrad writes dw [Co,Ci,3,3] and db [Co] (may be NULL).
 * linear: x [B,Fin], w [Fout,Fin], b [Fout], y [B,Fout].  The weight-gradient
 * calls split long reductions over several workgroups and take a 25 MB
 * stream-ordered workspace (hipMallocAsync / hipFreeAsync on the stream) for
 * the partial sums, which are added in a fixed order. */
int svr_conv3x3s2_forward(void* hip_stream, const float* x, const float* w, const float* b, float* y, int B,
                          int Ci, int H, int W, int Co, int relu);
int svr_conv3x3s2_dgrad(void* hip_stream, const float* dy, const float* y, const float* w, float* dx, int B,
                        int Ci, int H, int W, int Co);
int svr_conv3x3s2_wgrad(void* hip_stream, const float* dy, const float* y, const float* x, float* dw, float* db,
                        int B, int Ci, int H, int W, int Co);
int svr_linear_forward(void* hip_stream, const float* x, const float* w, const float* b, float* y, int B,
                       int Fin, int Fout, int relu);
int svr_linear_dgrad(void* hip_stream, const float* dy, const float* y, const float* w, float* dx, int B,
                     int Fin, int Fout);
int svr_linear_wgrad(void* hip_stream, const float* dy, const float* y, const float* x, float* dw, float* db,
                     int B, int Fin, int Fout);

#ifdef __cplusplus
}
#endif
#endif
