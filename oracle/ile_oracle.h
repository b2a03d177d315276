/*
 * ile_oracle.h -- plain FP64 CPU oracle for the ILE likelihood hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
 * binding may include, link or call this code; only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark do.  It shares no source
 * with the HIP path.
 *
 * Paper: Wysocki, O'Shaughnessy, Fang, Lange, "Accelerating parameter
 * inference with graphics processing units", arXiv:1902.04934.
 * Equation numbers below are the paper's printed numbering:
 *   (1) Gaussian-noise log-likelihood, (2) band-limited inner product,
 *   (4) marginalized likelihood, (5) complex strain, (6) mode expansion,
 *   (7) decomposed likelihood in Q, U, V, (8) definitions of Q, U, V,
 *   (9) time-marginalized likelihood, (10) matrix form.
 *
 * Parameter vector of one extrinsic sample (the order used everywhere):
 *   0 ra [rad], 1 dec [rad], 2 psi [rad], 3 phi [rad], 4 cos(iota),
 *   5 D [Mpc], 6 t_ref [s]
 */
#ifndef ILE_ORACLE_H
#define ILE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NPAR 7

typedef struct {
    int32_t n_det;
    int32_t n_lm;
    const int32_t *modes;   /* [n_lm][2] = (l, m) */
    double srate_hz;
    int32_t n_t;            /* odd number of time bins */
    double d_ref_mpc;
    double gmst_rad;
    double earth_radius_m;
    double t0_s;            /* time of Q[0] relative to the geocentre event time */
    int64_t n_q;
} orc_config;

typedef struct {
    double lat_deg, lon_deg, xarm_az_deg;
} orc_detector;

/* Sec. II.A (detector response below Eq. (6)): site vector r [m] and
 * detector tensor D = (x x^T - y y^T)/2 of an L-shaped interferometer. */
void orc_detector_frame(const orc_detector *det, double earth_radius_m,
                        double r[3], double D[9]);

/* Antenna patterns F+, Fx of detector tensor D for a source at (ra, dec)
 * with polarization angle psi, at Greenwich sidereal angle gmst. */
void orc_antenna(const double D[9], double ra, double dec, double psi,
                 double gmst, double *fplus, double *fcross);

/* Arrival delay at site r relative to the geocentre, tau = -n.r/c, with n
 * the unit vector towards the source. */
double orc_delay(const double r[3], double ra, double dec, double gmst);

/* Spin-weight -2 spherical harmonic -2Y_lm(theta, phi) (mode expansion,
 * Eq. (6)), Wigner-d closed form. */
void orc_sylm(int l, int m, double theta, double phi, double *re, double *im);

/* Unrounded window position x_k = (t_ref + tau_k - t0)/dt of every detector
 * for one sample; the window of detector k starts at Q index
 * floor(x_k + 1/2) - (n_t - 1)/2. */
void orc_window_position(const orc_config *cfg, const orc_detector *dets,
                         const double *theta, double *x_out);

/* ln L(theta, t_j) for j = 0..n_t-1, Eq. (7), with the window start indices
 * given explicitly in s_start (one per detector).  Returns 0, or -1 if a
 * window leaves [0, n_q). */
int orc_lnL_series_at(const orc_config *cfg, const double *Q, const double *U,
                      const double *V, const orc_detector *dets,
                      const double *theta, const int64_t *s_start,
                      double *lnL_out);

/* Same, with the window starts computed from the sample (nearest sample). */
int orc_lnL_series(const orc_config *cfg, const double *Q, const double *U,
                   const double *V, const orc_detector *dets,
                   const double *theta, double *lnL_out);

/* Eq. (9) on the bin grid: log((1/n_t) sum_j exp(lnL_j)). */
double orc_logmeanexp(const double *x, int64_t n);

/* ln L_margT for N samples given in SoA layout samples[7][N]; OpenMP over
 * samples.  Invalid samples (window outside Q, D <= 0, |cos iota| > 1)
 * give NaN.  Returns the number of invalid samples. */
int64_t orc_eval(const orc_config *cfg, const double *Q, const double *U,
                 const double *V, const orc_detector *dets,
                 const double *samples, int64_t n, double *out, int n_threads);

/* Importance-sampling reduction of Eq. (4) (Sec. II.A, II.C):
 *   ln w = lnLmargT + ln p - ln q,  ln L_marg = log(mean w),
 *   n_eff = sum w / max w, Kish = (sum w)^2 / sum w^2,
 *   sigma = sqrt(sum w^2/(sum w)^2 - 1/N)   (relative error of the mean).
 * Sums are accumulated in long double in index order. */
typedef struct {
    double ln_L_marg, n_eff, n_eff_kish, sigma, max_lnL;
    int64_t n_samples;
} orc_result;
void orc_integrate(const double *lnLmargT, const double *ln_p,
                   const double *ln_q, int64_t n, orc_result *res);

/* Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Prior draw of sample i from stream (seed, i): uniform ra, arcsine dec,
 * uniform psi in [0, pi), phi in [0, 2pi), cos iota in [-1, 1],
 * p(D) ~ D^2 on [d_min, d_max], uniform t_ref in [-t_ref_max, t_ref_max].
 * Writes samples[7][n] (SoA) and ln p (the prior density in these
 * coordinates). */
void orc_prior_draw(uint64_t seed, int64_t first, int64_t n, double d_min,
                    double d_max, double t_ref_max, double *samples,
                    int64_t ld, double *ln_p);

/* Plain adaptive sampler: histogram proposal in ra and sin(dec). */
void orc_hist_cdf(const double *P, int nb, double *C);
void orc_hist_draw(uint64_t seed, int64_t first, int64_t n, int nb,
                   const double *P_ra, const double *P_sd, double d_min,
                   double d_max, double t_ref_max, double *samples, int64_t ld,
                   double *ln_p, double *ln_q, int32_t *bins);
void orc_hist_refit(const int32_t *bins, int64_t ld, const double *lnw,
                    int64_t n, int nb, double floor_w, double scale,
                    double *P_ra, double *P_sd);

#ifdef __cplusplus
}
#endif
#endif
