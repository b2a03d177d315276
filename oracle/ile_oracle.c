/*
 * ile_oracle.c -- plain FP64 CPU oracle for the ILE likelihood hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; the product library never links it.  Built
 * with -O2 -ffp-contract=off and no fast-math so every operation rounds as
 * written.  Each function follows the passage of arXiv:1902.04934 named in
 * its comment; readings where the paper is silent or inconsistent are stated
 * where they are used.
 */
#include "ile_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_C_LIGHT 299792458.0

/* ---------------------------------------------------------------- geometry
 * Sec. II.A, below Eq. (6): h_k = F+ h+(t_k) + Fx hx(t_k).  The paper does
 * not spell out the antenna-pattern convention; this follows the standard
 * detector-tensor construction: site on a sphere of radius R, arms in the
 * local tangent plane, x-arm azimuth counted counter-clockwise from local
 * East, y-arm 90 degrees further, D = (x x^T - y y^T)/2. */
void orc_detector_frame(const orc_detector *det, double R, double r[3],
                        double D[9])
{
    double lat = det->lat_deg * ORC_PI / 180.0;
    double lon = det->lon_deg * ORC_PI / 180.0;
    double az = det->xarm_az_deg * ORC_PI / 180.0;
    double east[3] = {-sin(lon), cos(lon), 0.0};
    double north[3] = {-sin(lat) * cos(lon), -sin(lat) * sin(lon), cos(lat)};
    double x[3], y[3];
    for (int i = 0; i < 3; i++) {
        x[i] = cos(az) * east[i] + sin(az) * north[i];
        y[i] = cos(az + ORC_PI / 2.0) * east[i] + sin(az + ORC_PI / 2.0) * north[i];
    }
    r[0] = R * cos(lat) * cos(lon);
    r[1] = R * cos(lat) * sin(lon);
    r[2] = R * sin(lat);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            D[3 * i + j] = 0.5 * (x[i] * x[j] - y[i] * y[j]);
}

/* Polarization basis (X, Y) of a source at hour angle h = ra - gmst and
 * declination dec, rotated by psi; F+ = X.D.X - Y.D.Y, Fx = X.D.Y + Y.D.X. */
void orc_antenna(const double D[9], double ra, double dec, double psi,
                 double gmst, double *fplus, double *fcross)
{
    double h = ra - gmst;
    double eE[3] = {-sin(h), cos(h), 0.0};
    double eN[3] = {-sin(dec) * cos(h), -sin(dec) * sin(h), cos(dec)};
    double X[3], Y[3];
    for (int i = 0; i < 3; i++) {
        X[i] = -cos(psi) * eE[i] + sin(psi) * eN[i];
        Y[i] = sin(psi) * eE[i] + cos(psi) * eN[i];
    }
    double xdx = 0, ydy = 0, xdy = 0, ydx = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            xdx += X[i] * D[3 * i + j] * X[j];
            ydy += Y[i] * D[3 * i + j] * Y[j];
            xdy += X[i] * D[3 * i + j] * Y[j];
            ydx += Y[i] * D[3 * i + j] * X[j];
        }
    *fplus = xdx - ydy;
    *fcross = xdy + ydx;
}

/* Sec. II.A: arrival time t_k = t_c - x_k . n for a wave travelling along
 * n.  Read with n pointing to the source, a plane wave reaches a site at
 * r earlier by n.r/c than the geocentre, so tau = -n.r/c. */
double orc_delay(const double r[3], double ra, double dec, double gmst)
{
    double h = ra - gmst;
    double n[3] = {cos(dec) * cos(h), cos(dec) * sin(h), sin(dec)};
    double nr = n[0] * r[0] + n[1] * r[1] + n[2] * r[2];
    return -nr / ORC_C_LIGHT;
}

/* ------------------------------------------------------- -2Y_lm, Eq. (6)
 * Wigner-d form of the spin-weighted harmonic (Goldberg et al. 1967):
 *  -2Y_lm = sqrt((2l+1)/4pi) e^{i m phi} sum_k (-1)^k
 *     sqrt((l+m)!(l-m)!(l+2)!(l-2)!) / ((l+m-k)!(l-2-k)! k! (k+2-m)!)
 *     cos(theta/2)^{2l+m-2-2k} sin(theta/2)^{2k+2-m},
 *  k = max(0, m-2) .. min(l+m, l-2). */
static double orc_fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= (double)i;
    return f;
}

void orc_sylm(int l, int m, double theta, double phi, double *re, double *im)
{
    double c = cos(theta / 2.0), s = sin(theta / 2.0);
    int kmin = m - 2 > 0 ? m - 2 : 0;
    int kmax = (l + m) < (l - 2) ? (l + m) : (l - 2);
    double norm = sqrt(orc_fact(l + m) * orc_fact(l - m) * orc_fact(l + 2) *
                       orc_fact(l - 2));
    double sum = 0.0;
    for (int k = kmin; k <= kmax; k++) {
        double term = norm / (orc_fact(l + m - k) * orc_fact(l - 2 - k) *
                              orc_fact(k) * orc_fact(k + 2 - m));
        term *= pow(c, 2 * l + m - 2 - 2 * k) * pow(s, 2 * k + 2 - m);
        sum += (k % 2 == 0) ? term : -term;
    }
    double amp = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI)) * sum;
    *re = amp * cos(m * phi);
    *im = amp * sin(m * phi);
}

/* ------------------------------------------------------- time windows
 * Sec. II.A, after Eq. (9): Q_k,lm is a uniformly sampled series; sample
 * theta with reference time t_ref sees bin j (geocentre time
 * t_ref + (j - (n_t-1)/2) dt) at detector time t_ref + tau_k + ..., read at
 * the nearest sample of Q.  One rounding per (sample, detector). */
void orc_window_position(const orc_config *cfg, const orc_detector *dets,
                         const double *theta, double *x_out)
{
    double dt = 1.0 / cfg->srate_hz;
    for (int k = 0; k < cfg->n_det; k++) {
        double r[3], D[9];
        orc_detector_frame(&dets[k], cfg->earth_radius_m, r, D);
        double tau = orc_delay(r, theta[0], theta[1], cfg->gmst_rad);
        x_out[k] = (theta[6] + tau - cfg->t0_s) / dt;
    }
}

/* Eq. (7) (equivalently the matrix form Eq. (10)):
 *  ln L = (Dref/D) Re sum_k sum_lm (F_k Y_lm)^* Q_k,lm(t_k)
 *       - (Dref/D)^2/4 sum_k sum_{lm,l'm'} [ |F_k|^2 Y_lm^* Y_l'm' U_k
 *                                         + Re(F_k^2 Y_lm Y_l'm' V_k) ].
 * F_k = F+ + i Fx: with h = h+ - i hx (Eq. (5)) this is the sign for which
 * Eq. (7) equals Eq. (1); the sign printed next to Eq. (7) does not. */
static void orc_factors(const orc_config *cfg, const orc_detector *dets,
                        const double *theta, double *F /*[n_det][2]*/,
                        double *Y /*[n_lm][2]*/)
{
    for (int k = 0; k < cfg->n_det; k++) {
        double r[3], D[9], fp, fx;
        orc_detector_frame(&dets[k], cfg->earth_radius_m, r, D);
        orc_antenna(D, theta[0], theta[1], theta[2], cfg->gmst_rad, &fp, &fx);
        F[2 * k] = fp;
        F[2 * k + 1] = fx;
    }
    double iota = acos(theta[4]);
    for (int a = 0; a < cfg->n_lm; a++)
        orc_sylm(cfg->modes[2 * a], cfg->modes[2 * a + 1], iota, theta[3],
                 &Y[2 * a], &Y[2 * a + 1]);
}

int orc_lnL_series_at(const orc_config *cfg, const double *Q, const double *U,
                      const double *V, const orc_detector *dets,
                      const double *theta, const int64_t *s_start,
                      double *lnL_out)
{
    int nd = cfg->n_det, nl = cfg->n_lm;
    for (int k = 0; k < nd; k++)
        if (s_start[k] < 0 || s_start[k] + cfg->n_t > cfg->n_q) return -1;
    double *F = (double *)malloc(sizeof(double) * 2 * nd);
    double *Y = (double *)malloc(sizeof(double) * 2 * nl);
    orc_factors(cfg, dets, theta, F, Y);
    double kappa = cfg->d_ref_mpc / theta[5];

    /* quadratic term, independent of time */
    double quad = 0.0;
    for (int k = 0; k < nd; k++) {
        double fr = F[2 * k], fi = F[2 * k + 1];
        double f2abs = fr * fr + fi * fi;
        double f2r = fr * fr - fi * fi, f2i = 2.0 * fr * fi; /* F^2 */
        double uterm = 0.0, vr = 0.0, vi = 0.0;
        for (int a = 0; a < nl; a++)
            for (int b = 0; b < nl; b++) {
                const double *u = &U[2 * (((int64_t)k * nl + a) * nl + b)];
                const double *v = &V[2 * (((int64_t)k * nl + a) * nl + b)];
                double yar = Y[2 * a], yai = Y[2 * a + 1];
                double ybr = Y[2 * b], ybi = Y[2 * b + 1];
                /* conj(Y_a) Y_b */
                double cr = yar * ybr + yai * ybi, ci = yar * ybi - yai * ybr;
                uterm += cr * u[0] - ci * u[1];
                /* Y_a Y_b V_ab */
                double pr = yar * ybr - yai * ybi, pi = yar * ybi + yai * ybr;
                vr += pr * v[0] - pi * v[1];
                vi += pr * v[1] + pi * v[0];
            }
        quad += f2abs * uterm + (f2r * vr - f2i * vi);
    }
    quad *= kappa * kappa / 4.0;

    for (int j = 0; j < cfg->n_t; j++) {
        double lin = 0.0;
        for (int k = 0; k < nd; k++) {
            for (int a = 0; a < nl; a++) {
                /* c = kappa F_k Y_a; Re(conj(c) Q) */
                double fr = F[2 * k], fi = F[2 * k + 1];
                double yr = Y[2 * a], yi = Y[2 * a + 1];
                double cr = kappa * (fr * yr - fi * yi);
                double ci = kappa * (fr * yi + fi * yr);
                const double *q = &Q[2 * (((int64_t)k * nl + a) * cfg->n_q +
                                          s_start[k] + j)];
                lin += cr * q[0] + ci * q[1];
            }
        }
        lnL_out[j] = lin - quad;
    }
    free(F);
    free(Y);
    return 0;
}

static int orc_sample_valid(const double *theta)
{
    return theta[5] > 0.0 && theta[4] >= -1.0 && theta[4] <= 1.0;
}

int orc_lnL_series(const orc_config *cfg, const double *Q, const double *U,
                   const double *V, const orc_detector *dets,
                   const double *theta, double *lnL_out)
{
    int64_t s[64];
    double x[64];
    if (cfg->n_det > 64 || !orc_sample_valid(theta)) return -1;
    orc_window_position(cfg, dets, theta, x);
    for (int k = 0; k < cfg->n_det; k++) {
        double c = floor(x[k] + 0.5);
        if (!(c > -1e15 && c < 1e15)) return -1;
        s[k] = (int64_t)c - (cfg->n_t - 1) / 2;
    }
    return orc_lnL_series_at(cfg, Q, U, V, dets, theta, s, lnL_out);
}

/* Eq. (9) with T = n_t dt and the rectangle rule on the bin grid. */
double orc_logmeanexp(const double *x, int64_t n)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < n; i++)
        if (x[i] > m) m = x[i];
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += exp(x[i] - m);
    return m + log(s) - log((double)n);
}

int64_t orc_eval(const orc_config *cfg, const double *Q, const double *U,
                 const double *V, const orc_detector *dets,
                 const double *samples, int64_t n, double *out, int n_threads)
{
    int64_t bad = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads) reduction(+ : bad)
#endif
    {
        double *L = (double *)malloc(sizeof(double) * cfg->n_t);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t i = 0; i < n; i++) {
            double th[ORC_NPAR];
            for (int p = 0; p < ORC_NPAR; p++) th[p] = samples[p * n + i];
            if (orc_lnL_series(cfg, Q, U, V, dets, th, L) != 0) {
                out[i] = NAN;
                bad++;
            } else {
                out[i] = orc_logmeanexp(L, cfg->n_t);
            }
        }
        free(L);
    }
    return bad;
}

/* ------------------------------------------- importance-sampling reduction
 * Eq. (4) by Monte Carlo (Sec. II.A) with the accuracy measure of Sec. II.C.
 * The paper leaves n_eff = eps N_it undefined; read as sum w / max w. */
void orc_integrate(const double *lnLmargT, const double *ln_p,
                   const double *ln_q, int64_t n, orc_result *res)
{
    double M = -INFINITY, maxL = -INFINITY;
    for (int64_t i = 0; i < n; i++) {
        double lw = lnLmargT[i] + ln_p[i] - ln_q[i];
        if (lw > M) M = lw;
        if (lnLmargT[i] > maxL) maxL = lnLmargT[i];
    }
    res->n_samples = n;
    res->max_lnL = maxL;
    if (n == 0 || M == -INFINITY) {
        res->ln_L_marg = -INFINITY;
        res->n_eff = 0.0;
        res->n_eff_kish = 0.0;
        res->sigma = NAN;
        return;
    }
    long double s1 = 0.0L, s2 = 0.0L;
    for (int64_t i = 0; i < n; i++) {
        double lw = lnLmargT[i] + ln_p[i] - ln_q[i];
        long double e = expl((long double)lw - (long double)M);
        s1 += e;
        s2 += e * e;
    }
    res->ln_L_marg = (double)((long double)M + logl(s1) - logl((long double)n));
    res->n_eff = (double)s1;
    res->n_eff_kish = (double)(s1 * s1 / s2);
    long double var = s2 / (s1 * s1) - 1.0L / (long double)n;
    res->sigma = var > 0 ? (double)sqrtl(var) : 0.0;
}

/* ------------------------------------------------------------- Philox
 * Philox4x32 with 10 rounds as defined by Salmon et al. (SC'11): each round
 * multiplies counter words 0 and 2 by fixed odd constants, swaps and xors
 * the high halves with the other words and the key; the key is bumped by
 * the Weyl constants between rounds. */
static void orc_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        orc_mulhilo(0xD2511F53u, c[0], &hi0, &lo0);
        orc_mulhilo(0xCD9E8D57u, c[2], &hi1, &lo1);
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    memcpy(out, c, sizeof(c));
}

/* Stream layout shared by definition with the device sampler: sample i of
 * stream `seed` uses counters (i_lo, i_hi, b, 0x494C4531) for b = 0..3 under
 * key (seed_lo, seed_hi); parameter p takes words 2p and 2p+1 of the 16 and
 * forms the 53-bit uniform ((w0 >> 5) * 2^26 + (w1 >> 6) + 1/2) / 2^53. */
static double orc_u53(uint32_t w0, uint32_t w1)
{
    double a = (double)(w0 >> 5), b = (double)(w1 >> 6);
    return (a * 67108864.0 + b + 0.5) / 9007199254740992.0;
}

void orc_prior_draw(uint64_t seed, int64_t first, int64_t n, double d_min,
                    double d_max, double t_ref_max, double *samples,
                    int64_t ld, double *ln_p)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
    for (int64_t t = 0; t < n; t++) {
        uint64_t i = (uint64_t)(first + t);
        uint32_t w[16];
        for (uint32_t b = 0; b < 4; b++) {
            uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), b, 0x494C4531u};
            orc_philox4x32_10(ctr, key, &w[4 * b]);
        }
        double u[7];
        for (int p = 0; p < 7; p++) u[p] = orc_u53(w[2 * p], w[2 * p + 1]);
        double ra = 2.0 * ORC_PI * u[0];
        double dec = asin(2.0 * u[1] - 1.0);
        double psi = ORC_PI * u[2];
        double phi = 2.0 * ORC_PI * u[3];
        double ci = 2.0 * u[4] - 1.0;
        double D = cbrt(d_min * d_min * d_min + u[5] * v3);
        double tr = t_ref_max * (2.0 * u[6] - 1.0);
        samples[0 * ld + t] = ra;
        samples[1 * ld + t] = dec;
        samples[2 * ld + t] = psi;
        samples[3 * ld + t] = phi;
        samples[4 * ld + t] = ci;
        samples[5 * ld + t] = D;
        samples[6 * ld + t] = tr;
        if (ln_p) {
            ln_p[t] = -log(2.0 * ORC_PI) + log(cos(dec) / 2.0) - log(ORC_PI) -
                      log(2.0 * ORC_PI) - log(2.0) + log(3.0 * D * D / v3) -
                      log(2.0 * t_ref_max);
        }
    }
}

/* ------------------------------------------------- plain adaptive sampler
 * Sec. II.A cites an adaptive Monte Carlo and Sec. III.B says the sampling
 * prior is regenerated from the most recent chunk of points, in two sky
 * parameters; the paper gives no further detail.  Reading: the proposal is
 * a product of two nb-bin histogram densities, in ra on [0, 2 pi) and in
 * sin(dec) on [-1, 1], times the prior in the other five parameters.
 * Draws use the same counter-based uniforms as orc_prior_draw; ra and
 * sin(dec) go through the inverse CDF of the piecewise-constant density:
 * bin b is the last with C[b] <= u (C the running sum of P in bin order),
 * and the position inside it is (u - C[b]) / P[b]. */
static int orc_hist_invert(const double *P, const double *C, int nb, double u,
                           double *frac)
{
    int lo = 0, hi = nb - 1;     /* last b with C[b] <= u */
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (C[mid] <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    double f = (u - C[lo]) / P[lo];
    *frac = f < 1.0 ? f : 1.0;
    return lo;
}

void orc_hist_cdf(const double *P, int nb, double *C)
{
    C[0] = 0.0;
    for (int b = 0; b < nb; b++) C[b + 1] = C[b] + P[b];
}

void orc_hist_draw(uint64_t seed, int64_t first, int64_t n, int nb,
                   const double *P_ra, const double *P_sd, double d_min,
                   double d_max, double t_ref_max, double *samples, int64_t ld,
                   double *ln_p, double *ln_q, int32_t *bins)
{
    double *C_ra = (double *)malloc(sizeof(double) * (nb + 1));
    double *C_sd = (double *)malloc(sizeof(double) * (nb + 1));
    orc_hist_cdf(P_ra, nb, C_ra);
    orc_hist_cdf(P_sd, nb, C_sd);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
    for (int64_t t = 0; t < n; t++) {
        uint64_t i = (uint64_t)(first + t);
        uint32_t w[16];
        for (uint32_t b = 0; b < 4; b++) {
            uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), b, 0x494C4531u};
            orc_philox4x32_10(ctr, key, &w[4 * b]);
        }
        double u[7];
        for (int p = 0; p < 7; p++) u[p] = orc_u53(w[2 * p], w[2 * p + 1]);
        double fr, fs;
        int br = orc_hist_invert(P_ra, C_ra, nb, u[0], &fr);
        int bs = orc_hist_invert(P_sd, C_sd, nb, u[1], &fs);
        double ra = ((double)br + fr) * (2.0 * ORC_PI / nb);
        double sd = -1.0 + ((double)bs + fs) * (2.0 / nb);
        double dec = asin(sd);
        double psi = ORC_PI * u[2];
        double phi = 2.0 * ORC_PI * u[3];
        double ci = 2.0 * u[4] - 1.0;
        double D = cbrt(d_min * d_min * d_min + u[5] * v3);
        double tr = t_ref_max * (2.0 * u[6] - 1.0);
        samples[0 * ld + t] = ra;
        samples[1 * ld + t] = dec;
        samples[2 * ld + t] = psi;
        samples[3 * ld + t] = phi;
        samples[4 * ld + t] = ci;
        samples[5 * ld + t] = D;
        samples[6 * ld + t] = tr;
        double lp = -log(2.0 * ORC_PI) + log(cos(dec) / 2.0) - log(ORC_PI) -
                    log(2.0 * ORC_PI) - log(2.0) + log(3.0 * D * D / v3) -
                    log(2.0 * t_ref_max);
        /* q / p = (nb P_ra[br]) (nb P_sd[bs]) */
        double lq = lp + log(nb * P_ra[br]) + log(nb * P_sd[bs]);
        if (ln_p) ln_p[t] = lp;
        if (ln_q) ln_q[t] = lq;
        if (bins) {
            bins[t] = br;
            bins[ld + t] = bs;
        }
    }
    free(C_ra);
    free(C_sd);
}

/* Refit from the latest chunk: tempered weights w = exp(beta (ln w - max)),
 * beta = min(1, scale / (max - mean)) (the paper is silent on tempering;
 * this keeps a single sample from collapsing the proposal), bin sums in
 * sample order, then a mixture with the prior: P = (1 - floor) H / sum H +
 * floor / nb. */
void orc_hist_refit(const int32_t *bins, int64_t ld, const double *lnw,
                    int64_t n, int nb, double floor_w, double scale,
                    double *P_ra, double *P_sd)
{
    double M = -INFINITY, sum = 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (lnw[i] > M) M = lnw[i];
        sum += lnw[i];
    }
    double mean = sum / (double)n;
    double beta = (M - mean) > scale ? scale / (M - mean) : 1.0;
    long double *H = (long double *)calloc(2 * nb, sizeof(long double));
    long double tot = 0.0L;
    for (int64_t i = 0; i < n; i++) {
        double w = exp(beta * (lnw[i] - M));
        H[bins[i]] += w;
        H[nb + bins[ld + i]] += w;
        tot += w;
    }
    for (int b = 0; b < nb; b++) {
        P_ra[b] = (double)((1.0L - floor_w) * H[b] / tot) + floor_w / nb;
        P_sd[b] = (double)((1.0L - floor_w) * H[nb + b] / tot) + floor_w / nb;
    }
    free(H);
}
