/* FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see svr_oracle.h).
 *
 * Written from the paper in the world frame:
 *   O1  Gaussian j: R_j = rot(q/|q|) (Hamilton, w first), s = exp(log_scale),
 *       Sigma_j = R_j diag(s^2) R_j^T, det Sigma_j = prod s_k^2
 *       (Sec. 2.2, "Sigma = R S S^T R^T", log-space scales in the nomenclature).
 *   O2  Slice i: R_i = Exp(omega_i) R0_i, t_i = t0_i + tau_i (Sec. 2.1, 2.4),
 *       Sigma_PSF = diag((fwhm/2.355)^2) in the slice frame, rotated with the
 *       slice: P_i = R_i Sigma_PSF R_i^T (Sec. 2.3 Eq. 4, Sec. 2.4).
 *   O3  Pixel (row r, column k): u = ((k-(W-1)/2) dx, (r-(H-1)/2) dy, 0),
 *       x = R_i u + t_i (Eq. 1, T_i(u) = R_i u + t_i).
 *   O4  Sigma_obs = Sigma_j + P_i, d = x - mu_j, q = d^T Sigma_obs^-1 d,
 *       rho = sqrt(det Sigma_j / det Sigma_obs), value c_j rho w(exp(-q/2)).
 *   O5  y = sum over Gaussians of the pixel's subject.
 *
 * Pruning for a finite window tau (exact: skipped pairs contribute zero):
 *   the minimum of q over the slice plane is beta = (n.(mu-t))^2 / n^T Sigma_obs n;
 *   pairs with beta > tau^2 are skipped.  Otherwise, writing x* for the plane
 *   point reaching that minimum, q(x) = beta + (x-x*)^T Sigma_obs^-1 (x-x*) on the
 *   plane, which is >= beta + |x-x*|^2 / lambda_max >= beta + |x-x*|^2 / trace,
 *   so only pixels within radius sqrt((tau^2-beta) trace(Sigma_obs)) of x* are
 *   visited.
 *
 * Gradients (hand-derived, checked by central finite differences in tests),
 * per in-window pair with upstream g = dL/dy:
 *   w_e = g c rho e,  w_v = g c rho (e - e_tau),  L = Sigma_obs^-1
 *   dc      += g rho (e - e_tau)
 *   dmu     += w_e L d,         dx = -w_e L d
 *   G_obs   += 0.5 w_e (L d)(L d)^T - 0.5 w_v L   (dLoss = tr(G dSigma_obs))
 *   dlogs_k += w_v  (from sqrt det Sigma_j = exp(sum log s))
 *   then Sigma_obs = Sigma_j + P_i:  dlogs_k += 2 s_k^2 (R_j^T G R_j)_kk,
 *   dR_j = 2 G R_j diag(s^2), chained through the quaternion and its
 *   normalisation; pose: dtau += dx, left perturbation R <- Exp(delta) R gives
 *   ddelta += (R u) x dx + 2 (A12-A21, A20-A02, A01-A10) with A = P_i G,
 *   and d omega = J_l(omega)^T d delta (left Jacobian of SO(3)).
 */
#include "svr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FWHM_TO_SIGMA (1.0 / 2.355)

typedef struct {
    double R[9];      /* rotation, row-major */
    double S[9];      /* covariance */
    double s2[3];     /* squared scales */
    double det;       /* det Sigma_j */
    double qn[4];     /* normalised quaternion */
    double qlen;
} ora_gauss;

typedef struct {
    double R[9];
    double t[3];
    double P[9];      /* R Sigma_PSF R^T */
    double n[3];      /* slice normal (third column of R) */
    double dx, dy;
    int32_t H, W;
    int64_t off;
} ora_slice;

static void mat3_mul(const double* A, const double* B, double* C) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * a + k] * B[3 * k + b];
            C[3 * a + b] = s;
        }
}

static void mat3_transpose(const double* A, double* T) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) T[3 * a + b] = A[3 * b + a];
}

static double mat3_det(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse by the adjugate; returns the determinant */
static double mat3_inv(const double* A, double* Inv) {
    double det = mat3_det(A);
    double id = 1.0 / det;
    Inv[0] = (A[4] * A[8] - A[5] * A[7]) * id;
    Inv[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    Inv[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    Inv[3] = (A[5] * A[6] - A[3] * A[8]) * id;
    Inv[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    Inv[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    Inv[6] = (A[3] * A[7] - A[4] * A[6]) * id;
    Inv[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    Inv[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return det;
}

/* Hamilton quaternion (w,x,y,z), unit length, to a rotation matrix */
static void quat_to_rot(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void skew(const double* w, double* K) {
    K[0] = 0;     K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0;     K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0;
}

/* Rodrigues: Exp(w) = I + a K + b K^2, a = sin th / th, b = (1 - cos th)/th^2 */
static void so3_exp(const double* w, double* R) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), a, b;
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    double K[9], K2[9];
    skew(w, K);
    mat3_mul(K, K, K2);
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0 ? 1.0 : 0.0) + a * K[k] + b * K2[k];
}

/* Left Jacobian of SO(3): J = I + (1-cos th)/th^2 K + (th - sin th)/th^3 K^2 */
static void so3_left_jacobian(const double* w, double* J) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), b, c;
    if (th < 1e-4) {
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        c = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        b = (1.0 - cos(th)) / th2;
        c = (th - sin(th)) / (th2 * th);
    }
    double K[9], K2[9];
    skew(w, K);
    mat3_mul(K, K, K2);
    for (int k = 0; k < 9; ++k) J[k] = (k % 4 == 0 ? 1.0 : 0.0) + b * K[k] + c * K2[k];
}

static void setup_gauss(const ora_problem* p, int64_t j, ora_gauss* g) {
    const double* q = p->quat + 4 * j;
    double len = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    g->qlen = len;
    for (int k = 0; k < 4; ++k) g->qn[k] = q[k] / len;
    quat_to_rot(g->qn, g->R);
    double lsum = 0.0;
    for (int k = 0; k < 3; ++k) {
        double s = exp(p->log_scale[3 * j + k]);
        g->s2[k] = s * s;
        lsum += p->log_scale[3 * j + k];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += g->R[3 * a + k] * g->s2[k] * g->R[3 * b + k];
            g->S[3 * a + b] = v;
        }
    g->det = exp(2.0 * lsum);
}

static void setup_slice(const ora_problem* p, int32_t i, ora_slice* s) {
    double E[9];
    so3_exp(p->pose + 6 * i, E);
    mat3_mul(E, p->rot0 + 9 * i, s->R);
    for (int k = 0; k < 3; ++k) s->t[k] = p->trans0[3 * i + k] + p->pose[6 * i + 3 + k];
    double sig2[3];
    for (int k = 0; k < 3; ++k) {
        double sg = p->psf_fwhm[3 * i + k] * FWHM_TO_SIGMA;
        sig2[k] = sg * sg;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += s->R[3 * a + k] * sig2[k] * s->R[3 * b + k];
            s->P[3 * a + b] = v;
        }
    for (int k = 0; k < 3; ++k) s->n[k] = s->R[3 * k + 2];
    s->dx = p->spacing[2 * i];
    s->dy = p->spacing[2 * i + 1];
    s->H = p->height[i];
    s->W = p->width[i];
    s->off = p->pix_offset[i];
}

static void pixel_world(const ora_slice* s, int r, int k, double* x, double* Ru) {
    double u0 = (k - 0.5 * (s->W - 1)) * s->dx;
    double u1 = (r - 0.5 * (s->H - 1)) * s->dy;
    for (int a = 0; a < 3; ++a) {
        Ru[a] = s->R[3 * a] * u0 + s->R[3 * a + 1] * u1;
        x[a] = Ru[a] + s->t[a];
    }
}

typedef struct {
    double So[9];   /* Sigma_obs */
    double L[9];    /* inverse */
    double rho;
    int r0, r1, k0, k1;  /* inclusive pixel window */
    int keep;
} ora_pair;

static int is_finite_tau(double tau) { return tau > 0.0 && isfinite(tau); }

/* Pair set-up and pruning window */
static void setup_pair(const ora_gauss* g, const double* mu, const ora_slice* s, double tau,
                       ora_pair* pr) {
    for (int k = 0; k < 9; ++k) pr->So[k] = g->S[k] + s->P[k];
    double det = mat3_inv(pr->So, pr->L);
    pr->rho = sqrt(g->det / det);
    pr->keep = 1;
    pr->r0 = 0; pr->r1 = s->H - 1; pr->k0 = 0; pr->k1 = s->W - 1;
    if (!is_finite_tau(tau)) return;
    double dmt[3] = {mu[0] - s->t[0], mu[1] - s->t[1], mu[2] - s->t[2]};
    double nd = s->n[0] * dmt[0] + s->n[1] * dmt[1] + s->n[2] * dmt[2];
    double Sn[3];
    for (int a = 0; a < 3; ++a)
        Sn[a] = pr->So[3 * a] * s->n[0] + pr->So[3 * a + 1] * s->n[1] + pr->So[3 * a + 2] * s->n[2];
    double nSn = s->n[0] * Sn[0] + s->n[1] * Sn[1] + s->n[2] * Sn[2];
    double beta = nd * nd / nSn;
    if (beta > tau * tau) { pr->keep = 0; return; }
    double xs[3], us[2];
    for (int a = 0; a < 3; ++a) xs[a] = mu[a] - nd / nSn * Sn[a];
    /* slice-frame coordinates of x*: u = R^T (x* - t) */
    for (int b = 0; b < 2; ++b) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a) v += s->R[3 * a + b] * (xs[a] - s->t[a]);
        us[b] = v;
    }
    double tr = pr->So[0] + pr->So[4] + pr->So[8];
    double rad = sqrt((tau * tau - beta) * tr) * (1.0 + 1e-9) + 1e-9;
    double c0 = 0.5 * (s->W - 1), r0 = 0.5 * (s->H - 1);
    double kmin = ceil((us[0] - rad) / s->dx + c0), kmax = floor((us[0] + rad) / s->dx + c0);
    double rmin = ceil((us[1] - rad) / s->dy + r0), rmax = floor((us[1] + rad) / s->dy + r0);
    if (kmin < 0) kmin = 0;
    if (rmin < 0) rmin = 0;
    if (kmax > s->W - 1) kmax = s->W - 1;
    if (rmax > s->H - 1) rmax = s->H - 1;
    if (kmin > kmax || rmin > rmax) { pr->keep = 0; return; }
    pr->k0 = (int)kmin; pr->k1 = (int)kmax; pr->r0 = (int)rmin; pr->r1 = (int)rmax;
}

static double quad(const double* L, const double* d, double* Ld) {
    for (int a = 0; a < 3; ++a) Ld[a] = L[3 * a] * d[0] + L[3 * a + 1] * d[1] + L[3 * a + 2] * d[2];
    return d[0] * Ld[0] + d[1] * Ld[1] + d[2] * Ld[2];
}

static ora_gauss* make_gauss(const ora_problem* p) {
    ora_gauss* G = (ora_gauss*)malloc(sizeof(ora_gauss) * (size_t)(p->n_gauss > 0 ? p->n_gauss : 1));
    if (!G) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p->n_gauss; ++j) setup_gauss(p, j, &G[j]);
    return G;
}

static ora_slice* make_slices(const ora_problem* p) {
    ora_slice* S = (ora_slice*)malloc(sizeof(ora_slice) * (size_t)(p->n_slices > 0 ? p->n_slices : 1));
    if (!S) return NULL;
    for (int32_t i = 0; i < p->n_slices; ++i) setup_slice(p, i, &S[i]);
    return S;
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int ora_forward(const ora_problem* p, double tau, double* pred, int64_t* n_incut, int64_t* n_pairs) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    if (!G || !S) { free(G); free(S); return -1; }
    const int fin = is_finite_tau(tau);
    const double etau = fin ? exp(-0.5 * tau * tau) : 0.0;
    const double tau2 = fin ? tau * tau : INFINITY;
    int64_t cnt = 0, pairs = 0;
    memset(pred, 0, sizeof(double) * (size_t)p->pix_offset[p->n_slices]);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : cnt, pairs)
    for (int32_t i = 0; i < p->n_slices; ++i) {
        const ora_slice* s = &S[i];
        int32_t sub = p->slice_subject[i];
        for (int64_t j = p->gauss_offsets[sub]; j < p->gauss_offsets[sub + 1]; ++j) {
            const double* mu = p->mean + 3 * j;
            ora_pair pr;
            setup_pair(&G[j], mu, s, tau, &pr);
            if (!pr.keep) continue;
            ++pairs;
            double cr = p->amp[j] * pr.rho;
            for (int r = pr.r0; r <= pr.r1; ++r)
                for (int k = pr.k0; k <= pr.k1; ++k) {
                    double x[3], Ru[3], d[3], Ld[3];
                    pixel_world(s, r, k, x, Ru);
                    for (int a = 0; a < 3; ++a) d[a] = x[a] - mu[a];
                    double q = quad(pr.L, d, Ld);
                    if (q > tau2) continue;
                    pred[s->off + (int64_t)r * s->W + k] += cr * (exp(-0.5 * q) - etau);
                    ++cnt;
                }
        }
    }
    if (n_incut) *n_incut = cnt;
    if (n_pairs) *n_pairs = pairs;
    free(G);
    free(S);
    return 0;
}

static int32_t slice_of_pixel(const ora_problem* p, int64_t pix) {
    int32_t lo = 0, hi = p->n_slices - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (p->pix_offset[mid] <= pix) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int ora_forward_pixels(const ora_problem* p, double tau, int64_t n_sel, const int64_t* pix, double* out) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    if (!G || !S) { free(G); free(S); return -1; }
    const int fin = is_finite_tau(tau);
    const double etau = fin ? exp(-0.5 * tau * tau) : 0.0;
    const double tau2 = fin ? tau * tau : INFINITY;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = 0; e < n_sel; ++e) {
        int32_t i = slice_of_pixel(p, pix[e]);
        const ora_slice* s = &S[i];
        int64_t loc = pix[e] - s->off;
        int r = (int)(loc / s->W), k = (int)(loc % s->W);
        double x[3], Ru[3];
        pixel_world(s, r, k, x, Ru);
        int32_t sub = p->slice_subject[i];
        double acc = 0.0;
        for (int64_t j = p->gauss_offsets[sub]; j < p->gauss_offsets[sub + 1]; ++j) {
            const double* mu = p->mean + 3 * j;
            ora_pair pr;
            setup_pair(&G[j], mu, s, INFINITY, &pr);   /* no pruning */
            double d[3], Ld[3];
            for (int a = 0; a < 3; ++a) d[a] = x[a] - mu[a];
            double q = quad(pr.L, d, Ld);
            if (q > tau2) continue;
            acc += p->amp[j] * pr.rho * (exp(-0.5 * q) - etau);
        }
        out[e] = acc;
    }
    free(G);
    free(S);
    return 0;
}

/* Chain dLoss/dSigma_j (G, full symmetric matrix) and the direct sqrt(det)
 * term (wv) to the log-scales and the stored quaternion. */
static void chain_gauss(const ora_gauss* g, const double* Gsum, double wv_sum, double* gls_out,
                        double* gq_out) {
    /* Sigma_j = R diag(s^2) R^T */
    double Rt[9], RtG[9], RtGR[9];
    mat3_transpose(g->R, Rt);
    mat3_mul(Rt, Gsum, RtG);
    mat3_mul(RtG, g->R, RtGR);
    for (int k = 0; k < 3; ++k) gls_out[k] = wv_sum + 2.0 * g->s2[k] * RtGR[4 * k];
    double GR[9], dR[9];
    mat3_mul(Gsum, g->R, GR);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dR[3 * a + b] = 2.0 * GR[3 * a + b] * g->s2[b];
    double w = g->qn[0], x = g->qn[1], y = g->qn[2], z = g->qn[3];
    const double dRw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    const double dRx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    const double dRy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    const double dRz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    double gqn[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k) {
        gqn[0] += dR[k] * dRw[k];
        gqn[1] += dR[k] * dRx[k];
        gqn[2] += dR[k] * dRy[k];
        gqn[3] += dR[k] * dRz[k];
    }
    double dotp = gqn[0] * g->qn[0] + gqn[1] * g->qn[1] + gqn[2] * g->qn[2] + gqn[3] * g->qn[3];
    for (int k = 0; k < 4; ++k) gq_out[k] = (gqn[k] - g->qn[k] * dotp) / g->qlen;
}

/* Absolute contributions of one (pixel, Gaussian) pair to every gradient
 * component, added to bnd = [mean 3 | log_scale 3 | quat 4 | amp 1 | per-slice
 * pose 6*M] (pose rows start at offset 11).  Used for pairs whose inside/outside
 * decision lies within rounding of the cut. */
static void band_pair(const ora_gauss* g, const ora_slice* s, double gp, double c, double rho,
                      const double* L, const double* Ld, const double* Ru, double q, double etau,
                      double* bnd, int32_t slice) {
    double e = exp(-0.5 * q);
    double we = gp * c * rho * e;
    double wv = gp * c * rho * (e - etau);
    double Gp[9], gls[3], gq[4], A[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Gp[3 * a + b] = 0.5 * we * Ld[a] * Ld[b] - 0.5 * wv * L[3 * a + b];
    chain_gauss(g, Gp, wv, gls, gq);
    double dx[3] = {-we * Ld[0], -we * Ld[1], -we * Ld[2]};
    mat3_mul(s->P, Gp, A);
    double pd[3] = {Ru[1] * dx[2] - Ru[2] * dx[1] + 2.0 * (A[5] - A[7]),
                    Ru[2] * dx[0] - Ru[0] * dx[2] + 2.0 * (A[6] - A[2]),
                    Ru[0] * dx[1] - Ru[1] * dx[0] + 2.0 * (A[1] - A[3])};
    for (int a = 0; a < 3; ++a) bnd[a] += fabs(we * Ld[a]);
    for (int a = 0; a < 3; ++a) bnd[3 + a] += fabs(gls[a]);
    for (int a = 0; a < 4; ++a) bnd[6 + a] += fabs(gq[a]);
    bnd[10] += fabs(gp * rho * (e - etau));
    /* pose: |d delta| in the left-perturbation frame and |d tau| */
    for (int a = 0; a < 3; ++a) {
        bnd[11 + 6 * slice + a] += fabs(pd[a]);
        bnd[11 + 6 * slice + 3 + a] += fabs(dx[a]);
    }
}

/* Per-Gaussian gradient over all its slices; pose contributions are added to
 * gpose_delta/gpose_tau ([M,3] each) when non-NULL. */
static void gauss_backward(const ora_problem* p, const ora_gauss* G, const ora_slice* S, int64_t j,
                           double tau, const double* grad_pred, double* gmu_out, double* gls_out,
                           double* gq_out, double* gc_out, double* gdelta, double* gtau,
                           double band, double* bnd) {
    const int fin = is_finite_tau(tau);
    const double etau = fin ? exp(-0.5 * tau * tau) : 0.0;
    const double tau2 = fin ? tau * tau : INFINITY;
    const double* mu = p->mean + 3 * j;
    const double c = p->amp[j];
    const ora_gauss* g = &G[j];
    double Gsum[9] = {0}, gmu[3] = {0}, gc = 0.0, wv_sum = 0.0;
    int32_t sub = -1;
    for (int32_t sb = 0; sb < p->n_subjects; ++sb)
        if (j >= p->gauss_offsets[sb] && j < p->gauss_offsets[sb + 1]) { sub = sb; break; }
    for (int32_t i = 0; i < p->n_slices; ++i) {
        if (p->slice_subject[i] != sub) continue;
        const ora_slice* s = &S[i];
        ora_pair pr;
        setup_pair(g, mu, s, bnd ? tau * sqrt(1.0 + band) : tau, &pr);
        if (!pr.keep) continue;
        double Gij[9] = {0}, ptau[3] = {0}, pdel[3] = {0};
        for (int r = pr.r0; r <= pr.r1; ++r)
            for (int k = pr.k0; k <= pr.k1; ++k) {
                double gp = grad_pred[s->off + (int64_t)r * s->W + k];
                if (gp == 0.0) continue;
                double x[3], Ru[3], d[3], Ld[3];
                pixel_world(s, r, k, x, Ru);
                for (int a = 0; a < 3; ++a) d[a] = x[a] - mu[a];
                double q = quad(pr.L, d, Ld);
                if (bnd && fabs(q - tau2) <= band * tau2) {
                    band_pair(g, s, gp, c, pr.rho, pr.L, Ld, Ru, q, etau, bnd, i);
                    continue;
                }
                if (q > tau2) continue;
                double e = exp(-0.5 * q);
                double we = gp * c * pr.rho * e;
                double wv = gp * c * pr.rho * (e - etau);
                gc += gp * pr.rho * (e - etau);
                wv_sum += wv;
                double dxv[3];
                for (int a = 0; a < 3; ++a) {
                    gmu[a] += we * Ld[a];
                    dxv[a] = -we * Ld[a];
                    ptau[a] += dxv[a];
                }
                pdel[0] += Ru[1] * dxv[2] - Ru[2] * dxv[1];
                pdel[1] += Ru[2] * dxv[0] - Ru[0] * dxv[2];
                pdel[2] += Ru[0] * dxv[1] - Ru[1] * dxv[0];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        Gij[3 * a + b] += 0.5 * we * Ld[a] * Ld[b] - 0.5 * wv * pr.L[3 * a + b];
            }
        for (int k = 0; k < 9; ++k) Gsum[k] += Gij[k];
        if (gdelta) {
            double A[9];
            mat3_mul(s->P, Gij, A);
            pdel[0] += 2.0 * (A[5] - A[7]);
            pdel[1] += 2.0 * (A[6] - A[2]);
            pdel[2] += 2.0 * (A[1] - A[3]);
            for (int a = 0; a < 3; ++a) {
                gdelta[3 * i + a] += pdel[a];
                gtau[3 * i + a] += ptau[a];
            }
        }
    }
    chain_gauss(g, Gsum, wv_sum, gls_out, gq_out);
    for (int a = 0; a < 3; ++a) gmu_out[a] = gmu[a];
    *gc_out = gc;
}

int ora_backward(const ora_problem* p, double tau, const double* grad_pred, double* g_mean,
                 double* g_log_scale, double* g_quat, double* g_amp, double* g_pose) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    int32_t M = p->n_slices;
    double* dsum = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
    if (!G || !S || !dsum) { free(G); free(S); free(dsum); return -1; }
#pragma omp parallel
    {
        double* dloc = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
        double* gdel = dloc;
        double* gtau = dloc + 3 * (size_t)M;
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < p->n_gauss; ++j)
            gauss_backward(p, G, S, j, tau, grad_pred, g_mean + 3 * j, g_log_scale + 3 * j,
                           g_quat + 4 * j, g_amp + j, gdel, gtau, 0.0, NULL);
#pragma omp critical
        for (size_t k = 0; k < (size_t)M * 6; ++k) dsum[k] += dloc[k];
        free(dloc);
    }
    for (int32_t i = 0; i < M; ++i) {
        double J[9];
        so3_left_jacobian(p->pose + 6 * i, J);
        const double* dd = dsum + 3 * i;
        for (int a = 0; a < 3; ++a)
            g_pose[6 * i + a] = J[a] * dd[0] + J[3 + a] * dd[1] + J[6 + a] * dd[2];  /* J^T dd */
        for (int a = 0; a < 3; ++a) g_pose[6 * i + 3 + a] = dsum[3 * (size_t)M + 3 * i + a];
    }
    free(dsum);
    free(G);
    free(S);
    return 0;
}

int ora_backward_subset(const ora_problem* p, double tau, const double* grad_pred, int64_t n_sel,
                        const int64_t* gauss_idx, double* g_mean, double* g_log_scale,
                        double* g_quat, double* g_amp) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    if (!G || !S) { free(G); free(S); return -1; }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = 0; e < n_sel; ++e)
        gauss_backward(p, G, S, gauss_idx[e], tau, grad_pred, g_mean + 3 * e, g_log_scale + 3 * e,
                       g_quat + 4 * e, g_amp + e, NULL, NULL, 0.0, NULL);
    free(G);
    free(S);
    return 0;
}

/* Band-split gradient: pairs with |q - tau^2| <= band * tau^2 are left out of
 * the gradient and their absolute contributions are summed into b_* instead
 * (b_pose in the (omega, tau) parameterisation, bounded through |J_l^T|).  Any
 * gradient that decides those pairs either way lies within g +- b. */
int ora_backward_band(const ora_problem* p, double tau, double band, const double* grad_pred,
                      double* g_mean, double* g_log_scale, double* g_quat, double* g_amp,
                      double* g_pose, double* b_mean, double* b_log_scale, double* b_quat,
                      double* b_amp, double* b_pose) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    int32_t M = p->n_slices;
    size_t nb = 11 + 6 * (size_t)M;
    double* dsum = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
    double* bpose = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
    if (!G || !S || !dsum || !bpose) { free(G); free(S); free(dsum); free(bpose); return -1; }
#pragma omp parallel
    {
        double* dloc = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
        double* bloc = (double*)calloc(nb, sizeof(double));
        double* bpl = (double*)calloc((size_t)M * 6 + 6, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < p->n_gauss; ++j) {
            memset(bloc, 0, 11 * sizeof(double));
            gauss_backward(p, G, S, j, tau, grad_pred, g_mean + 3 * j, g_log_scale + 3 * j,
                           g_quat + 4 * j, g_amp + j, dloc, dloc + 3 * (size_t)M, band, bloc);
            for (int a = 0; a < 3; ++a) { b_mean[3 * j + a] = bloc[a]; b_log_scale[3 * j + a] = bloc[3 + a]; }
            for (int a = 0; a < 4; ++a) b_quat[4 * j + a] = bloc[6 + a];
            b_amp[j] = bloc[10];
            for (size_t k = 0; k < (size_t)M * 6; ++k) { bpl[k] += bloc[11 + k]; bloc[11 + k] = 0.0; }
        }
#pragma omp critical
        {
            for (size_t k = 0; k < (size_t)M * 6; ++k) { dsum[k] += dloc[k]; bpose[k] += bpl[k]; }
        }
        free(dloc);
        free(bloc);
        free(bpl);
    }
    for (int32_t i = 0; i < M; ++i) {
        double J[9];
        so3_left_jacobian(p->pose + 6 * i, J);
        const double* dd = dsum + 3 * i;
        for (int a = 0; a < 3; ++a)
            g_pose[6 * i + a] = J[a] * dd[0] + J[3 + a] * dd[1] + J[6 + a] * dd[2];
        for (int a = 0; a < 3; ++a) g_pose[6 * i + 3 + a] = dsum[3 * (size_t)M + 3 * i + a];
        const double* bd = bpose + 6 * (size_t)i;
        for (int a = 0; a < 3; ++a)
            b_pose[6 * i + a] = fabs(J[a]) * bd[0] + fabs(J[3 + a]) * bd[1] + fabs(J[6 + a]) * bd[2];
        for (int a = 0; a < 3; ++a) b_pose[6 * i + 3 + a] = bd[3 + a];
    }
    free(dsum);
    free(bpose);
    free(G);
    free(S);
    return 0;
}

/* Band-split forward: pred_core excludes pairs with |q - tau^2| <= band * tau^2,
 * b_pred sums their |value|. */
int ora_forward_band(const ora_problem* p, double tau, double band, double* pred_core, double* b_pred) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    if (!G || !S) { free(G); free(S); return -1; }
    const double etau = exp(-0.5 * tau * tau);
    const double tau2 = tau * tau;
    memset(pred_core, 0, sizeof(double) * (size_t)p->pix_offset[p->n_slices]);
    memset(b_pred, 0, sizeof(double) * (size_t)p->pix_offset[p->n_slices]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < p->n_slices; ++i) {
        const ora_slice* s = &S[i];
        int32_t sub = p->slice_subject[i];
        for (int64_t j = p->gauss_offsets[sub]; j < p->gauss_offsets[sub + 1]; ++j) {
            const double* mu = p->mean + 3 * j;
            ora_pair pr;
            setup_pair(&G[j], mu, s, tau * sqrt(1.0 + band), &pr);
            if (!pr.keep) continue;
            double cr = p->amp[j] * pr.rho;
            for (int r = pr.r0; r <= pr.r1; ++r)
                for (int k = pr.k0; k <= pr.k1; ++k) {
                    double x[3], Ru[3], d[3], Ld[3];
                    pixel_world(s, r, k, x, Ru);
                    for (int a = 0; a < 3; ++a) d[a] = x[a] - mu[a];
                    double q = quad(pr.L, d, Ld);
                    int64_t pix = s->off + (int64_t)r * s->W + k;
                    double v = cr * (exp(-0.5 * q) - etau);
                    if (fabs(q - tau2) <= band * tau2) b_pred[pix] += fabs(v);
                    else if (q < tau2) pred_core[pix] += v;
                }
        }
    }
    free(G);
    free(S);
    return 0;
}

/* Band-split gradient for a subset of Gaussians (no pose output). */
int ora_backward_subset_band(const ora_problem* p, double tau, double band, const double* grad_pred,
                             int64_t n_sel, const int64_t* gauss_idx, double* g_mean,
                             double* g_log_scale, double* g_quat, double* g_amp, double* b_mean,
                             double* b_log_scale, double* b_quat, double* b_amp) {
    ora_gauss* G = make_gauss(p);
    ora_slice* S = make_slices(p);
    if (!G || !S) { free(G); free(S); return -1; }
    size_t nb = 11 + 6 * (size_t)p->n_slices;
    int fail = 0;
#pragma omp parallel
    {
        double* bloc = (double*)calloc(nb, sizeof(double));
        if (!bloc) fail = 1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t e = 0; e < n_sel; ++e) {
            if (!bloc) continue;
            memset(bloc, 0, nb * sizeof(double));
            gauss_backward(p, G, S, gauss_idx[e], tau, grad_pred, g_mean + 3 * e, g_log_scale + 3 * e,
                           g_quat + 4 * e, g_amp + e, NULL, NULL, band, bloc);
            for (int a = 0; a < 3; ++a) { b_mean[3 * e + a] = bloc[a]; b_log_scale[3 * e + a] = bloc[3 + a]; }
            for (int a = 0; a < 4; ++a) b_quat[4 * e + a] = bloc[6 + a];
            b_amp[e] = bloc[10];
        }
        free(bloc);
    }
    free(G);
    free(S);
    return fail ? -1 : 0;
}
