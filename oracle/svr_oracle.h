/* FP64 CPU oracle for the Gaussian-primitive slice acquisition model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; it exists so that tests, the smoke check and the CPU-baseline
 * leg of the benchmark can compare the GPU path against a plain, slow and
 * obviously correct evaluation written straight from the paper.
 *
 * Model (Sec. 2.1 Eq. 1, Sec. 2.3 Eqs. 3-5, with the sqrt(det) amplitude that
 * makes the covariance-addition result equal to the acquisition integral):
 *
 *   y_i(u) = sum_j c_j * rho_ij * w(e_ij(u)),
 *   Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T            (Eq. 4)
 *   rho_ij    = sqrt(det Sigma_j / det Sigma_obs)
 *   e_ij(u)   = exp(-0.5 d^T Sigma_obs^-1 d),  d = T_i(u) - mu_j
 *   w(e)      = e                       (tau = infinity: exact model)
 *   w(e)      = max(e - exp(-tau^2/2), 0)  (tau finite: continuous 3-sigma window)
 *
 * Everything is evaluated in the world frame, in double precision.
 * All arrays are host arrays in double (int32/int64 where noted).
 */
#ifndef SVR_ORACLE_H
#define SVR_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n_gauss;
    const double* mean;        /* [N,3] mm */
    const double* log_scale;   /* [N,3] s = exp(log_scale) mm */
    const double* quat;        /* [N,4] (w,x,y,z), any nonzero length */
    const double* amp;         /* [N] */
    int32_t n_subjects;
    const int64_t* gauss_offsets;  /* [S+1] */
    int32_t n_slices;
    const int32_t* slice_subject;  /* [M] */
    const int32_t* height;         /* [M] rows */
    const int32_t* width;          /* [M] columns */
    const int64_t* pix_offset;     /* [M+1] */
    const double* rot0;        /* [M,9] row-major */
    const double* trans0;      /* [M,3] */
    const double* pose;        /* [M,6] omega (rad), tau (mm) */
    const double* spacing;     /* [M,2] dx (columns), dy (rows) mm */
    const double* psf_fwhm;    /* [M,3] mm, slice frame */
} ora_problem;

/* Full forward: pred[P] (overwritten).  n_incut / n_pairs may be NULL.
 * n_incut counts (pixel, Gaussian) pairs with q <= tau^2 (all pairs when tau is
 * infinite); n_pairs counts (slice, Gaussian) pairs whose plane test passes. */
int ora_forward(const ora_problem* p, double tau, double* pred,
                int64_t* n_incut, int64_t* n_pairs);

/* Forward at selected global pixel indices only (no pruning, every Gaussian of
 * the pixel's subject is visited). */
int ora_forward_pixels(const ora_problem* p, double tau, int64_t n_sel,
                       const int64_t* pix, double* out);

/* Gradient of sum_p grad_pred[p] * y[p] with respect to every parameter.
 * Outputs are overwritten.  g_pose [M,6] = (d/d omega, d/d tau). */
int ora_backward(const ora_problem* p, double tau, const double* grad_pred,
                 double* g_mean, double* g_log_scale, double* g_quat,
                 double* g_amp, double* g_pose);

/* Same gradient for a subset of Gaussians only (rows of the outputs are the
 * subset order); pose gradients are not produced. */
int ora_backward_subset(const ora_problem* p, double tau, const double* grad_pred,
                        int64_t n_sel, const int64_t* gauss_idx,
                        double* g_mean, double* g_log_scale, double* g_quat,
                        double* g_amp);

/* Band-split variants: pairs whose q lies within band * tau^2 of the cut are
 * excluded from the result and their absolute contributions are reported
 * separately, component by component.  Any evaluation that decides those
 * pairs either way (e.g. in lower precision) lies within result +- bound. */
int ora_backward_band(const ora_problem* p, double tau, double band, const double* grad_pred,
                      double* g_mean, double* g_log_scale, double* g_quat, double* g_amp,
                      double* g_pose, double* b_mean, double* b_log_scale, double* b_quat,
                      double* b_amp, double* b_pose);
int ora_forward_band(const ora_problem* p, double tau, double band, double* pred_core,
                     double* b_pred);
int ora_backward_subset_band(const ora_problem* p, double tau, double band, const double* grad_pred,
                             int64_t n_sel, const int64_t* gauss_idx, double* g_mean,
                             double* g_log_scale, double* g_quat, double* g_amp, double* b_mean,
                             double* b_log_scale, double* b_quat, double* b_amp);

int ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
