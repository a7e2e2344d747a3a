/*
 * dnb_orbitfit.h -- orbit fit of a stream progenitor and its Fisher matrix
 * (libdnb.so; arXiv 2511.22468, Sec. 2.2.2 "Orbit fitting and Fisher contours").
 *
 * Only the progenitor is evolved, as one test particle: from its present-day
 * phase-space point it is integrated forward and backward in time in the host
 * potential (NFW halo + Miyamoto-Nagai disk, the same accelerations as dnb.h)
 * with n_steps kick-drift-kick steps of dt_total / n_steps each way.  The orbit
 * is compared with a stream track through
 *     chi2(p) = sum_k sum_c ((y_c(phi1_k; p) - y_c,k) / sigma_c)^2,
 * the paper's log-likelihood up to a factor.  The free parameters are the five
 * host-potential parameters in dex:
 *     p = log10(M_NFW, rs_NFW, M_MN, a_MN, b_MN)       (M_NFW: NFW scale mass).
 *
 * Observables.  The paper's GD-1 frame and data are not used; the orbit is
 * expressed in the orbit-aligned frame of the present-day point (e1 along x_now,
 * n along x_now x v_now, e2 = n x e1):
 *     phi1 = longitude in the (e1, e2) plane, continuous along the orbit, 0 at
 *            t = 0 (accumulated from the per-step turning angles, each step must
 *            turn by less than 90 degrees),
 *     y_0 = phi2 = asin(x.n / |x|) [rad],  y_1 = d = |x| [kpc],
 *     y_2 = v_r = x.v / |x| [km/s].
 * A track point k is (phi1_k, phi2_k, d_k, v_r,k); the model value at phi1_k is
 * the linear interpolation along phi1 on the first orbit segment, in time order
 * from t = 0, whose phi1 interval holds phi1_k: forward branch for phi1_k >= 0,
 * backward branch otherwise.  A point that no segment reaches makes chi2 = +inf.
 *
 * Conventions are those of dnb.h (device pointers unless "host", asynchronous
 * on `stream`, host-side argument checks returning DNB_ERR_ARG before anything
 * is enqueued).  Every array is FP64.  A track holds 1 <= K <= DNB_TRACK_MAX
 * points; batch <= DNB_BATCH_MAX.
 */
#ifndef DNB_ORBITFIT_H
#define DNB_ORBITFIT_H

#include "dnb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DNB_TRACK_MAX 64

typedef struct dnb_track_model {
    double w_now[6];   /* present-day (x, y, z, vx, vy, vz) of the progenitor */
    double G;          /* gravitational constant, > 0 */
    double dt_total;   /* time span of each branch, > 0 */
    int64_t n_steps;   /* steps per branch, >= 1 */
    double sigma[3];   /* errors of phi2 [rad], d [kpc], v_r [km/s], > 0 */
} dnb_track_model;

/* Model observables at the longitudes phi1 [K] for the parameters p [5]:
 * y [K][3] = (phi2, d, v_r) per point (+inf where unreached).  For mock tracks. */
dnb_status dnb_track_observe(dnb_ctx* ctx, const dnb_track_model* model, int64_t K,
                             const double* phi1, const double* p, double* y, void* stream);

/* chi2 of every parameter vector p [batch][5] against track [K][4] (rows
 * phi1, phi2, d, v_r): chi2 [batch]; jtr [batch][5] = J^T r and jtj [batch][15]
 * = J^T J (upper triangle, row by row), both nullable, with r the normalised
 * residuals and J = dr/dp from forward-mode derivatives through the integrator. */
dnb_status dnb_track_chi2(dnb_ctx* ctx, const dnb_track_model* model, int64_t K,
                          const double* track, int64_t batch, const double* p, double* chi2,
                          double* jtr, double* jtj, void* stream);

/* Exact Hessian hess [batch][5][5] = d2 chi2 / dp dp (second-order forward
 * derivatives through the integrator; within the current interpolation
 * segments) and, if cov is not NULL, the covariance cov [batch][5][5] = F^-1 of
 * the Fisher matrix F = hess / 2 (Sec. 2.2.2), NaN where F is not positive
 * definite.  Units: dex. */
dnb_status dnb_track_hessian(dnb_ctx* ctx, const dnb_track_model* model, int64_t K,
                             const double* track, int64_t batch, const double* p, double* hess,
                             double* cov, void* stream);

/* Levenberg-Marquardt from many starts (Sec. 2.2.2: the least-squares fit is
 * started from many sampled parameter vectors and the lowest chi2 kept).  p
 * [batch][5] holds the starts on entry and the fits on return; chi2 [batch]
 * the final chi2.  Each start takes n_iter iterations of: solve
 * (J^T J + lam diag(J^T J)) delta = -J^T r, accept p + delta if chi2 decreases
 * (lam /= 10, floor 1e-12), else keep p (lam *= 10, cap 1e16); lam starts at
 * lambda0 > 0.  A start with an infinite chi2 stays where it is.  Uses the
 * context's workspace: one call at a time per context. */
dnb_status dnb_track_lm(dnb_ctx* ctx, const dnb_track_model* model, int64_t K,
                        const double* track, int64_t batch, double* p, int64_t n_iter,
                        double lambda0, double* chi2, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DNB_ORBITFIT_H */
