/*
 * ile.h -- C ABI of libile, the MI355X (gfx950) implementation of the
 * extrinsic-marginalized likelihood of RIFT's ILE step, after Wysocki,
 * O'Shaughnessy, Fang and Lange, "Accelerating parameter inference with
 * graphics processing units", arXiv:1902.04934, Sec. II.A-II.C.
 *
 * For one intrinsic point the caller supplies the precomputed inner-product
 * series Q_k,lm(t) and the mode-overlap matrices U_k, V_k of Eq. (8); for a
 * block of extrinsic samples theta_alpha the library evaluates Eq. (7) on a
 * grid of n_t time bins, marginalizes over time (Eq. (9)) and reduces the
 * importance-weighted samples to ln L_marg (Eq. (4)) and n_eff (Sec. II.C).
 * Around that path: Q, U, V built on the device from frequency-domain
 * series (ile_set_data_fd, Eq. (2) and Eq. (8)); the adaptive and learned
 * samplers (ile_run) with reuse from one intrinsic point to the next; the
 * batched form for many points (ile_batch_*); joint extrinsic posterior
 * draws from a final iteration (ile_harvest_dev, Sec. V); and the surrogate
 * form, one Monte Carlo over intrinsic and extrinsic parameters
 * (ile_rom_*, Sec. V).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sample layout: SoA double samples[7][N], parameter rows
 *   0 ra [rad], 1 dec [rad], 2 psi [rad], 3 phi [rad], 4 cos(iota),
 *   5 D [Mpc], 6 t_ref [s]  (bin-grid centre, geocentre time).
 * Detector response: F_k = F+ + i Fx with the antenna patterns of an
 *   L-shaped detector (x-arm azimuth counted counter-clockwise from local
 *   East, y-arm 90 degrees further, spherical Earth of radius
 *   earth_radius_m); the paper prints F+ - i Fx beside Eq. (7), but only
 *   F+ + i Fx makes Eq. (7) equal Eq. (1) for h = h+ - i hx (Eq. (5)).
 * Harmonics: -2Y_lm(iota, phi) in the Wigner-d form; modes are any (l, m)
 *   with 2 <= l <= 6, |m| <= l.
 * Time: Q[i] is the value at detector time t0 + i/srate (t0 given at
 *   set_data).  Sample alpha and bin j (0 <= j < n_t, n_t odd) mean the
 *   geocentre time t_ref + (j - (n_t-1)/2)/srate; detector k reads
 *   Q_k,lm[s_k + j] with s_k = floor((t_ref + tau_k - t0) srate + 1/2)
 *   - (n_t-1)/2 and tau_k = -n.r_k/c (n towards the source).
 * Likelihood per bin (Eq. (7)):
 *   L_alpha,j = sum_k Re sum_lm conj(c_k,lm) Q_k,lm[s_k + j] - q_alpha,
 *   c_k,lm = (d_ref/D) F_k Y_lm,
 *   q_alpha = (d_ref/D)^2/4 sum_k [ |F_k|^2 Y^H U_k Y + Re(F_k^2 Y^T V_k Y) ].
 * Time marginalization (Eq. (9)) with T = n_t/srate, rectangle rule:
 *   lnLmargT_alpha = log( (1/n_t) sum_j exp(L_alpha,j) ).
 * Importance sampling (Eq. (4), Sec. II.C): ln w = lnLmargT + ln p - ln q,
 *   ln_L_marg = log(mean w), n_eff = sum w / max w,
 *   n_eff_kish = (sum w)^2 / sum w^2,
 *   sigma_ln_L = sqrt(sum w^2 / (sum w)^2 - 1/N)  (relative error of mean w).
 *
 * Precision: FP64 evaluates everything in double.  FP32 and BF16 run the
 * bulk Q contraction in float (BF16: hi/lo bfloat16 split of Q and of the
 * coefficients on the matrix cores, float accumulation); the quadratic term,
 * the time log-sum-exp and the sample reduction stay in double.
 *
 * Ownership and threading: the caller owns every buffer it passes; the
 * library copies Q/U/V at set_data and keeps no caller pointer.  A context
 * owns its device memory and one stream (the caller's, if given).  A
 * context is not thread-safe; distinct contexts are independent.
 *
 * Errors: every entry point returns an ile_status; nothing throws or aborts
 * across the ABI.  Host-pointer entry points leave outputs untouched on
 * error.  Device-pointer (_dev) entry points are asynchronous on the
 * context's stream: invalid samples there produce NaN outputs and a sticky
 * ILE_E_RANGE that ile_sync reports.  ile_last_error gives a message for the
 * last failing call on that context (valid until the next call on it).
 */
#ifndef ILE_H
#define ILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ile_ctx ile_ctx;
typedef struct ile_prop ile_prop;   /* learned proposal, below */

typedef enum {
    ILE_OK = 0,
    ILE_E_ARG = 1,         /* bad argument (null pointer, size, even n_t ...) */
    ILE_E_STATE = 2,       /* call out of order (eval before set_data)         */
    ILE_E_RANGE = 3,       /* sample or window outside its declared range     */
    ILE_E_NUMERIC = 4,     /* non-finite Q/U/V, or U not Hermitian            */
    ILE_E_DEVICE = 5,      /* HIP runtime error or no usable GPU              */
    ILE_E_NOMEM = 6,       /* device allocation failed                        */
    ILE_E_UNSUPPORTED = 7  /* valid request the library does not support      */
} ile_status;

typedef enum { ILE_FP64 = 0, ILE_FP32 = 1, ILE_BF16 = 2 } ile_precision;

typedef struct {
    double lat_deg, lon_deg, xarm_az_deg;
} ile_detector;

typedef struct {
    int32_t l, m;
} ile_mode;

#define ILE_MAX_DET 4
#define ILE_MAX_LM 32

typedef struct {
    int32_t n_det;            /* 1 .. ILE_MAX_DET                            */
    int32_t n_lm;             /* 1 .. ILE_MAX_LM                             */
    const ile_mode *modes;    /* [n_lm], copied                              */
    double srate_hz;          /* sampling rate of Q                          */
    int32_t n_t;              /* odd number of time bins, 1 .. 65535         */
    double d_ref_mpc;         /* fiducial distance of Eq. (6)                */
    double gmst_rad;          /* Greenwich sidereal angle (F time-independent) */
    double earth_radius_m;    /* site radius                                 */
    double t_ref_max_s;       /* |t_ref| bound checked at eval               */
    ile_precision precision;  /* bulk contraction precision                  */
    int32_t device;           /* HIP device ordinal                          */
    void *stream;             /* hipStream_t to use, or NULL for a new one   */
} ile_config;

typedef struct {
    double ln_L_marg;
    double n_eff;
    double n_eff_kish;
    double sigma_ln_L;
    double max_ln_L;          /* max over samples of lnLmargT                */
    int64_t n_samples;
} ile_result;

/* Create a context (allocates nothing large).  Fails with ILE_E_ARG on a
 * bad config, ILE_E_DEVICE when no GPU is usable.  *out is NULL on error. */
ile_status ile_create(const ile_config *cfg, ile_ctx **out);

/* Q: host double [n_det][n_lm][n_q][2] (re, im); U, V: host double
 * [n_det][n_lm][n_lm][2]; dets: [n_det].  t0_s: time of Q[0] relative to
 * the geocentre event time.  Copies the data to the device (converting Q to
 * the context precision).  ILE_E_NUMERIC if anything is non-finite or U_k
 * is not Hermitian to 1e-12 relative; ILE_E_RANGE if a sample with
 * |t_ref| <= t_ref_max could read outside [0, n_q). */
ile_status ile_set_data(ile_ctx *ctx, const double *Q, int64_t n_q,
                        double t0_s, const double *U, const double *V,
                        const ile_detector *dets);

/* Q, U, V of Eq. (8) built on the device from frequency-domain series and
 * installed as by ile_set_data.  Each inner product is Eq. (2) as a sum over
 * the n_q-point FFT grid f_i = i df for i < n_q/2, else (i - n_q) df:
 *   <a|b>_k   = 2 df sum_{f_min < |f_i| < f_max} conj(a_i) b_i / S_k,i,
 *   Q_k,lm[s] = 2 df sum_i exp(2 pi i f_i t_s) conj(h_lm,i) d_k,i / S_k,i
 *               over the same band, t_s = t0_s + s / (n_q df),
 *   U_k = <h_lm|h_l'm'>_k,   V_k = <h*_lm|h_l'm'>_k, whose summand is
 *               h_lm,-i h_l'm',i / S_k,i (the transform of conj(h) at f is
 *               conj(h(-f))).
 * h_f: host double [n_lm][n_q][2], the modes' transforms (time origin at
 * the geocentre event time); d_f: host double [n_det][n_q][2], the data's
 * transforms on the same clock; psd: host double [n_det][n_q], S_k at
 * |f_i|, positive and finite inside the band.  The band is open; f_min < 0
 * includes f = 0.  Q takes one inverse FFT per (detector, mode) row on the
 * device (FP64; in LDS, the four-step form above 1024 points).  n_q must be a power of two in
 * [2, 2^20] (ILE_E_UNSUPPORTED otherwise).  Q_out, U_out, V_out (may be
 * NULL) receive host copies in ile_set_data's layouts.  Errors:
 * ILE_E_ARG for NULL inputs, df <= 0, f_max <= f_min or a non-finite t0_s;
 * ILE_E_NUMERIC for a non-finite input or a bad spectrum in the band; then
 * ile_set_data's checks. */
ile_status ile_set_data_fd(ile_ctx *ctx, const double *h_f, const double *d_f,
                           const double *psd, int64_t n_q, double df, double f_min,
                           double f_max, double t0_s, const ile_detector *dets,
                           double *Q_out, double *U_out, double *V_out);

/* The same construction on device buffers, without installing: h_f_dev
 * [n_lm][n_q][2], d_f_dev [n_det][n_q][2], psd_dev [n_det][n_q] in; Q_dev
 * [n_det][n_lm][n_q][2], U_dev and V_dev [n_det][n_lm][n_lm][2] out (every
 * buffer the caller's).  Blocking; ile_last_kernel_ms then gives the inverse
 * FFT's device time.  Errors as ile_set_data_fd. */
ile_status ile_qvu_fd_dev(ile_ctx *ctx, const double *h_f_dev, const double *d_f_dev,
                          const double *psd_dev, int64_t n_q, double df, double f_min,
                          double f_max, double t0_s, double *Q_dev, double *U_dev,
                          double *V_dev);

/* A zero-noise injection built on the device and installed as by
 * ile_set_data: a physically consistent instance for tests of recovery.
 * White unit-variance noise, so Eq. (2) is <a|b> = sum_i conj(a_i) b_i with
 * circular shifts.  From mode series h_lm (host double [n_lm][n_q][2]) and
 * injected parameters theta[7]:
 *   d_k[i]   = Re(F_k (D_ref/D) sum_lm Y_lm h_lm[(i - lag_k) mod n_q]),
 *              F_k = F+ + i Fx, lag_k = floor((t_ref + tau_k - t0)/dt + 1/2),
 *   Q_k,lm[s] = sum_i conj(h_lm[(i - s) mod n_q]) d_k[i]        (Eq. (8)),
 *   U_k = sum_i conj(h_a[i]) h_b[i],  V_k = sum_i h_a[i] h_b[i]  (every k).
 * If snr > 0 the data are scaled to network SNR sqrt(sum_k <d_k|d_k>) =
 * snr, which moves the injected distance to *d_inj_out.  rho2_out (SNR^2),
 * d_inj_out and the host copies Q_out, U_out, V_out (layouts of
 * ile_set_data) may be NULL. */
ile_status ile_inject(ile_ctx *ctx, const double *h_lm, int64_t n_q, double t0_s,
                      const ile_detector *dets, const double *theta, double snr,
                      double *rho2_out, double *d_inj_out, double *Q_out, double *U_out,
                      double *V_out);

/* ln L_margT for N host samples into host lnL_margT[N].  ILE_E_RANGE if any
 * sample has D <= 0, |cos iota| > 1, |t_ref| > t_ref_max or a non-finite
 * value (message names the first).  N = 0 is a no-op. */
ile_status ile_eval(ile_ctx *ctx, const double *samples, int64_t N,
                    double *lnL_margT);

/* Eval plus the importance-sampling reduction; ln_p and ln_q are host
 * double [N] (log prior and log proposal density of each sample). */
ile_status ile_integrate(ile_ctx *ctx, const double *samples,
                         const double *ln_p, const double *ln_q, int64_t N,
                         ile_result *out);

/* Debug: the per-bin values L_alpha,j into host lnL[N][n_t]; same kernels
 * as ile_eval. */
ile_status ile_eval_series(ile_ctx *ctx, const double *samples, int64_t N,
                           double *lnL);

/* Device-pointer forms of the above (stream-ordered, asynchronous).
 * ile_integrate_dev writes the 6 result fields as doubles to the device
 * buffer result_dev[6] (n_samples as a double). */
ile_status ile_eval_dev(ile_ctx *ctx, const double *samples_dev, int64_t N,
                        double *lnL_margT_dev);
ile_status ile_integrate_dev(ile_ctx *ctx, const double *samples_dev,
                             const double *ln_p_dev, const double *ln_q_dev,
                             int64_t N, double *result_dev);

/* Allocation-free form of ile_integrate_dev, for callers that cannot
 * allocate device memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and result as ile_integrate_dev; the call itself allocates
 * nothing (no hipMalloc, hipFree, event or library allocation): its
 * workspace (per-sample lnL, window starts, sort keys and order, the
 * per-sample terms of Eq. (7), bucket counts, reduction partials) is a fixed
 * array of about 55 MiB that every GPU the library runs on holds until the
 * process ends, located in ile_create.  N <= ILE_NOALLOC_MAX_N, else
 * ILE_E_ARG and nothing runs.  The array is shared by every context and call on one GPU and keeps the
 * last call's contents (each call clears what must start at zero): calls
 * that overlap on one GPU (contexts on different streams) race; calls on
 * one stream are ordered.  A range error of a device-side sample is
 * reported by ile_sync, as for ile_integrate_dev.  The contraction's kernel
 * time is not recorded (ile_last_kernel_ms is unchanged). */
#define ILE_NOALLOC_MAX_N 65536
ile_status ile_integrate_dev_noalloc(ile_ctx *ctx, const double *samples_dev,
                                     const double *ln_p_dev, const double *ln_q_dev,
                                     int64_t N, double *result_dev);

/* Device prior draw (Philox4x32-10, Salmon et al. SC'11): sample i of
 * stream `seed` uses counters (i mod 2^32, i / 2^32, b, 0x494C4531), b =
 * 0..3, key (seed mod 2^32, seed / 2^32); parameter p takes words 2p, 2p+1
 * and forms the 53-bit uniform ((w0>>5) 2^26 + (w1>>6) + 1/2) 2^-53.
 * Prior: ra, psi, phi uniform; sin(dec), cos(iota) uniform; p(D) ~ D^2 on
 * [d_min, d_max]; t_ref uniform in [-t_ref_max, t_ref_max].  Writes device
 * samples_dev[7][ld] (columns first .. first+N-1 of the stream go to
 * columns 0 .. N-1) and ln_p_dev[N] (may be NULL). */
ile_status ile_draw_prior_dev(ile_ctx *ctx, uint64_t seed, int64_t first,
                              int64_t N, double d_min, double d_max,
                              double *samples_dev, int64_t ld,
                              double *ln_p_dev);

/* Whole hot path on the device: draw N prior samples (as ile_draw_prior_dev
 * with first = 0) in chunks of `chunk`, evaluate, reduce; only the result
 * crosses to the host.  chunk <= 0 means one chunk. */
ile_status ile_run_prior(ile_ctx *ctx, uint64_t seed, int64_t N,
                         int64_t chunk, double d_min, double d_max,
                         ile_result *out);

/* ------------------------------------------- surrogate (linear-basis) form
 * One Monte Carlo over intrinsic and extrinsic parameters at once (Sec. V:
 * a linear representation of h_lm through basis functions gives the
 * likelihood as a function of both).  The templates are
 *   h_lm(lambda; t) = sum_b c_lm,b(lambda) e_b(t),
 *   c_lm,b(lambda)  = sum_p A[lm][b][p] lambda^p,   lambda in [-1, 1],
 * so by linearity of Eq. (2), with C = [c_lm,b]:
 *   Q_k,lm(t) = sum_b conj(c_lm,b) Q^B_k,b(t),  U_k = conj(C) G_k C^T,
 *   V_k = C H_k C^T,
 * where Q^B_k,b(t) = <e_b(t)|d>_k, G_k = <e_b|e_b'>_k, H_k = <e_b*|e_b'>_k.
 * Usage: create the context with n_lm = the basis size (its mode list is not
 * used for harmonics in this form; any valid list), install Q^B, G, H as Q,
 * U, V (ile_set_data or ile_set_data_fd), then ile_rom_set.  Eq. (7) then
 * holds with -2Y_lm replaced by z_b = sum_lm c_lm,b(lambda) -2Y_lm(iota, phi)
 * of the physical modes, computed per sample on the device.
 *
 * ile_rom_set: modes [n_lm] the physical modes (as in ile_config, n_lm <=
 * ILE_MAX_LM), n_pow in [1, 8] powers of lambda, A host double
 * [n_lm][n_b][n_pow][2] (n_b = the context's n_lm), copied.  ILE_E_ARG for a
 * bad mode or size, ILE_E_NUMERIC for a non-finite A.
 * ile_rom_eval_dev / ile_rom_integrate_dev: as ile_eval_dev and
 * ile_integrate_dev for joint samples samples_dev[8][N]: rows 0..6 as
 * everywhere, row 7 lambda.  A lambda outside [-1, 1] gives a NaN output
 * and the sticky ILE_E_RANGE of ile_sync; ILE_E_STATE before ile_rom_set.
 * Plain evaluation (ile_eval and the rest) of the same context keeps using
 * its own mode list's harmonics. */
ile_status ile_rom_set(ile_ctx *ctx, const ile_mode *modes, int32_t n_lm, int32_t n_pow,
                       const double *A);
ile_status ile_rom_eval_dev(ile_ctx *ctx, const double *samples_dev, int64_t N,
                            double *lnL_margT_dev);
ile_status ile_rom_integrate_dev(ile_ctx *ctx, const double *samples_dev,
                                 const double *ln_p_dev, const double *ln_q_dev,
                                 int64_t N, double *result_dev);

/* ------------------------------------------------- extrinsic harvest
 * Joint extrinsic posterior draws from one final Monte Carlo iteration
 * (Sec. V: joint intrinsic and extrinsic information harvested from a
 * single final iteration; Eq. (3) at fixed intrinsic parameters).  The N
 * device samples samples_dev[7][N] with log prior ln_p_dev[N] and log
 * proposal density ln_q_dev[N] (either may be NULL: 0) and the bin grid of
 * Eq. (9) carry the joint weight exp(ln p_alpha - ln q_alpha + L_alpha,j).
 * Draw k (0 <= k < n_out) takes
 *   alpha_k = the first alpha whose cumulative weight (index order) exceeds
 *             u[0][k] times the total, the weight being
 *             exp(lnLmargT_alpha + ln p_alpha - ln q_alpha), Eq. (4);
 *   j_k     = the first bin whose cumulative exp(L_alpha_k,j) exceeds
 *             u[1][k] times that sample's total,
 * and when rounding leaves the target at the total, the first index that
 * reaches it (an index of zero weight is never drawn).  u_dev is device
 * double [2][n_out] of uniforms in [0, 1), the caller's random numbers.
 * Writes device idx_dev[n_out] (alpha_k), bin_dev[n_out] (j_k) and, if
 * theta_dev is not NULL, theta_dev[7][n_out]: sample alpha_k with row 6
 * replaced by the bin's geocentre time t_ref + (j_k - (n_t-1)/2)/srate.
 * If result_dev is not NULL it receives the Eq. (4) reduction of the same
 * evaluation, as ile_integrate_dev writes it (6 doubles), so that one call
 * is the whole final iteration: ln L_marg and the joint draws.
 * ln p = -inf is a zero weight.  Blocking (returns when the outputs are
 * written).  Errors: ILE_E_ARG for N <= 0, n_out < 0 or a NULL pointer
 * that is needed; ILE_E_RANGE for a sample out of range (as ile_eval), a
 * NaN ln p or ln q, ln p = +inf, ln q = -inf, or a uniform outside
 * [0, 1); ILE_E_NUMERIC if no sample has a finite positive weight.  On
 * error the outputs are unspecified.  Device work: one evaluation of the N
 * samples, then the per-bin series of the drawn samples in chunks of at
 * most 2 GiB, kept by the context for reuse (n_out = 0 is a no-op). */
ile_status ile_harvest_dev(ile_ctx *ctx, const double *samples_dev,
                           const double *ln_p_dev, const double *ln_q_dev,
                           int64_t N, const double *u_dev, int64_t n_out,
                           int64_t *idx_dev, int32_t *bin_dev,
                           double *theta_dev, double *result_dev);

/* ----------------------------------------------------------- samplers
 * The Monte Carlo over extrinsic parameters (Sec. II.A: direct Monte Carlo
 * with an adaptive sampling prior; Sec. III.B: the sampling prior is
 * regenerated from the most recent chunk of points, in two sky parameters).
 *
 * Plain adaptive sampler: the proposal is a product of two n_bins-bin
 * histogram densities, in ra on [0, 2 pi) and in sin(dec) on [-1, 1], times
 * the prior in the other five parameters.  Draws use the Philox stream of
 * ile_draw_prior_dev (same counters and uniforms); ra and sin(dec) go
 * through the inverse CDF of the histograms (bin b = last with C[b] <= u,
 * C the running sum of P in bin order; position (u - C[b]) / P[b]).
 * ln q = ln p + ln(n_bins P_ra[b_ra]) + ln(n_bins P_sd[b_sd]).
 * A refit from a chunk tempers its weights, w = exp(beta (ln w - max)) with
 * beta = min(1, temper / (max ln w - mean ln w)), sums them per bin, and
 * mixes with the prior: P = (1 - floor) H / sum H + floor / n_bins.  Every
 * sum runs in a fixed order (bit-reproducible).  The context holds the
 * current histograms (initially uniform = the prior). */
#define ILE_MAX_BINS 64

typedef enum {
    ILE_SAMPLER_PRIOR = 0,     /* proposal = prior (ln p - ln q = 0)        */
    ILE_SAMPLER_ADAPTIVE = 1,  /* histogram proposal, refit per chunk       */
    ILE_SAMPLER_LEARNED = 2    /* adaptive rounds, then the learned proposal */
} ile_sampler;

typedef struct {
    ile_sampler sampler;
    uint64_t seed;           /* Philox key; sample i of the run uses counter i */
    int64_t chunk;           /* samples per chunk (<= 0: 100000)             */
    int64_t max_samples;     /* hard stop (> 0)                              */
    double n_eff_target;     /* stop once n_eff >= target (<= 0: never)      */
    double d_min_mpc, d_max_mpc;  /* distance prior support                  */
    int32_t n_bins;          /* bins per adapted parameter (<= 0: 50)        */
    double floor;            /* prior weight in each refit (< 0: 0.1)        */
    double temper;           /* tempering scale (<= 0: 10)                   */
    int32_t adapt_chunks;    /* refit after at most this many chunks; < 0:
                                until ln L_marg > max(10, max lnLmargT / 2) */
    int32_t reset;           /* 1: start from uniform histograms; 0: keep the
                                context's current ones (warm start)          */
    /* sampler LEARNED only: adapt_chunks (<= 0: 3) adaptive rounds of
     * `chunk` samples fill a training ring of as many chunks and train
     * `prop` (train_steps Adam steps of train_batch, learning rate lr;
     * <= 0: 300, 16384, 2e-3).  Refinement: chunks are drawn from
     * (1 - eps) q_net + eps q_hist (the histograms as left by the rounds);
     * each replaces the oldest chunk of the ring and the network is refit
     * (transform and refine_steps warm Adam steps), until a chunk's own
     * n_eff reaches refine_eff times its size or refine_rounds refits are
     * spent.  Then a probe chunk of the mixture: if its n_eff is below
     * fallback_neff, it becomes one more refinement chunk while refits
     * remain, and refinement resumes; with none left the run continues
     * with the adaptive sampler.  Then chunks are drawn until n_eff_target
     * or max_samples.  The estimate covers the chunks after the last probe
     * only (refinement chunks and probes are never part of it). */
    ile_prop *prop;
    double eps;              /* defensive weight (< 0: 0.1)                   */
    double fallback_neff;    /* (< 0: 1000; 0: never fall back)               */
    int32_t train_steps, train_batch;
    double lr;
    int32_t refine_rounds;   /* refits after the first training (< 0: 24)     */
    int32_t refine_steps;    /* (<= 0: 150)                                   */
    double refine_eff;       /* (<= 0: 0.05)                                  */
    double train_ess;        /* tempering target of the training weights, as
                                ess_frac of ile_prop_train_opts (<= 0: 0.01) */
    double refine_kish;      /* also stop refining once a chunk's Kish size
                                (sum w)^2 / sum w^2 reaches this fraction of
                                it (<= 0: no such test, the default: a Kish
                                size can look healthy while the n_eff of the
                                chunks after it is not)                       */
    double sigma_scale;      /* kappa set on prop for the refinement and
                                estimation draws (<= 0: 1.2)                 */
    int32_t warm;            /* sampler LEARNED: 1 = prop carries a network
                                trained at another intrinsic point (the
                                integrator reused from point to point, Sec.
                                II.C): the adaptive rounds draw from its
                                defensive mixture (with the context's
                                histograms, which are not refit in them)
                                instead of from the histograms, and the first
                                training takes refine_steps warm Adam steps
                                from its current weights.  0: as described
                                above                                        */
} ile_run_opts;

/* Monte Carlo estimate of ln L_marg: chunk after chunk, draw on the device,
 * evaluate, accumulate the mergeable partials (M, S1, S2, n); refit the
 * adaptive proposal after each of the first chunks; stop at n_eff_target
 * or max_samples.  Each chunk's weights use the proposal it was drawn from,
 * so the combined estimate is unbiased.  n_chunks_out may be NULL. */
ile_status ile_run(ile_ctx *ctx, const ile_run_opts *opts, ile_result *out,
                   int64_t *n_chunks_out);

/* Result of the last ile_run with sampler LEARNED: samples of each phase,
 * whether it fell back, training time and the last refinement efficiency. */
typedef struct {
    int64_t n_train_samples;   /* adaptive rounds                            */
    int64_t n_refine_samples;  /* refinement chunks                          */
    int64_t n_learned_samples; /* estimation chunks from the mixture         */
    int32_t fell_back;
    double train_ms;           /* device time of all training steps          */
    double final_loss;
    double last_refine_eff;    /* n_eff / n of the last refinement chunk     */
    double refine_eff[32];     /* n_eff / n of refinement chunks 0..31       */
    double refine_kish[32];    /* Kish size / n of refinement chunks 0..31  */
} ile_learned_info;
ile_status ile_last_learned_info(const ile_ctx *ctx, ile_learned_info *out);

/* Copy the context's histograms out / in (host arrays of n_bins doubles;
 * ile_hist_set normalizes nothing: P must be positive and sum to 1). */
ile_status ile_hist_get(ile_ctx *ctx, int32_t n_bins, double *P_ra, double *P_sd);
ile_status ile_hist_set(ile_ctx *ctx, int32_t n_bins, const double *P_ra,
                        const double *P_sd);

/* Device draw from the context's histograms: samples_dev[7][ld], ln_p_dev,
 * ln_q_dev [N] (either may be NULL), bins_dev int32 [2][ld] (ra bin, sin
 * dec bin; may be NULL). */
ile_status ile_hist_draw_dev(ile_ctx *ctx, uint64_t seed, int64_t first, int64_t N,
                             double d_min, double d_max, double *samples_dev,
                             int64_t ld, double *ln_p_dev, double *ln_q_dev,
                             int32_t *bins_dev);

/* Device refit of the context's histograms from N samples given by their
 * bins (int32 [2][ld]) and log-weights lnLmargT + ln p - ln q (ln_p_dev and
 * ln_q_dev may be NULL = 0). */
ile_status ile_hist_refit_dev(ile_ctx *ctx, const int32_t *bins_dev, int64_t ld,
                              const double *lnL_dev, const double *ln_p_dev,
                              const double *ln_q_dev, int64_t N, double floor,
                              double temper);

/* --------------------------------------------------- learned proposal
 * Not in the paper, which adapts 1-D histograms (Sec. II.A, Sec. III.C): a
 * masked autoregressive mixture density network over the 7 extrinsic
 * parameters, trained on the weighted samples of the first adaptive rounds
 * and used in a defensive mixture with the histogram proposal.
 *
 * Transform x -> z~ (x in the sample order ra, dec, psi, phi, cos iota, D,
 * t_ref): u = frac((x - origin)/P + 1/2) for ra (P = 2 pi), psi (P = pi),
 * phi (P = 2 pi); u = (sin dec + 1)/2, (cos iota + 1)/2, (D - d_min)/(d_max
 * - d_min), (t_ref + t_max)/(2 t_max); z = ln(u/(1-u)); z~ = (z - mean) /
 * scale.  ln q(x) = ln q(z~) + sum_d ln |dz~_d/dx_d| (-inf if a u is 0 or 1).
 *
 * Network: h1 = tanh(W1 z~ + b1), h2 = tanh(W2 h1 + b2), o = W3 h2 + b3;
 * float32 parameters, ILE_PROP_NPARAM of them, flat and row-major:
 *   W1[128][7] | b1[128] | W2[128][128] | b2[128] | W3[336][128] | b3[336].
 * MADE masks, hidden degree deg(k) = k mod 6: W1[k][i] used iff i <= deg(k),
 * W2[k2][k1] iff deg(k1) <= deg(k2), W3[o][k] iff deg(k) < o / 48; masked
 * entries are held at zero.  Dimension d is a 16-component Gaussian mixture
 * in z~_d with logits o[48d + c], means o[48d + 16 + c] and scales
 * kappa (sigma_floor + softplus(o[48d + 32 + c])): kappa (sigma_scale, 1
 * by default) widens every component when drawing and evaluating ln q, an
 * exact density of its own; training always fits the kappa = 1 model.
 *
 * Device arithmetic: layer 1 FP32; layers 2 and 3 BF16 on the matrix cores
 * with FP32 accumulation; mixture densities FP32; transform, Jacobian,
 * ln p and the defensive mixture FP64.  Draws: Philox4x32-10 counters
 * (i, b, 0x4D444E31), b = 0..7, key seed: uniforms 0..6 choose components,
 * 7..14 give normals (Box-Muller), 15 picks the member of the defensive
 * mixture; a histogram member draws exactly as ile_hist_draw_dev (counter
 * i).  The ln q returned by ile_prop_sample_dev is bit-identical to what
 * ile_prop_logpdf_dev returns for the drawn sample.
 *
 * Training minimizes -sum w ln q(z~) / sum w with Adam (0.9, 0.999, 1e-8)
 * on minibatches drawn from the training set with probability proportional
 * to the tempered weights w = exp(beta (ln w - max)) over the finite ln w:
 * beta = 1 if the Kish effective size (sum w)^2 / sum w^2 reaches
 * max(1, ess_frac * count), else the largest beta (30 halvings of [0, 1])
 * that reaches it.  Each workgroup's gradient is one partial row, summed in
 * a fixed order, so training is bit-reproducible. */
#define ILE_PROP_NPARAM 60880

typedef struct {
    double d_min_mpc, d_max_mpc, t_ref_max_s;   /* prior support            */
    double sigma_floor;      /* <= 0: 1e-3                                    */
    uint64_t seed;           /* initial weights                               */
    int32_t device;
    void *stream;            /* hipStream_t, or NULL for a new one            */
    double sigma_scale;      /* kappa of the draws and densities (<= 0: 1)    */
} ile_prop_config;

typedef struct {
    int32_t steps;           /* Adam steps (<= 0: 1000)                       */
    int32_t batch;           /* minibatch (<= 0: 4096)                        */
    double lr;               /* (<= 0: 1e-3)                                  */
    double ess_frac;         /* tempering target, fraction of the samples
                                (<= 0: 0.01)                                  */
    uint64_t seed;           /* minibatch draws                               */
    int32_t fit_transform;   /* 1: fit the transform to the data first:
                                weighted circular means of ra, psi, phi as
                                origins, weighted mean / standard deviation
                                of z (>= 1e-3) as mean / scale            */
} ile_prop_train_opts;

ile_status ile_prop_create(const ile_prop_config *cfg, ile_prop **out);
/* Host float32 arrays of ILE_PROP_NPARAM values (set: masked entries are
 * zeroed, Adam state reset). */
ile_status ile_prop_set_params(ile_prop *p, const float *params);
ile_status ile_prop_get_params(ile_prop *p, float *params);
ile_status ile_prop_set_transform(ile_prop *p, const double origin[3], const double mean[7],
                                  const double scale[7]);
ile_status ile_prop_get_transform(ile_prop *p, double origin[3], double mean[7],
                                  double scale[7]);
/* kappa > 0 for the following draws and densities (ILE_E_ARG otherwise). */
ile_status ile_prop_set_sigma_scale(ile_prop *p, double kappa);
/* Fit the transform to device samples x_dev[7][ld] with log-weights
 * lnw_dev, tempered as for training (ess_frac <= 0: 0.01). */
ile_status ile_prop_fit_transform_dev(ile_prop *p, const double *x_dev, int64_t ld,
                                      const double *lnw_dev, int64_t n, double ess_frac);
/* Loss -sum w ln q(z~) / sum w of n device samples (w_dev NULL: all 1) and
 * its gradient (device float grad_dev[ILE_PROP_NPARAM], may be NULL; masked
 * entries 0); loss to the host (may be NULL).  n <= 2^20. */
ile_status ile_prop_grad_dev(ile_prop *p, const double *x_dev, int64_t ld, const double *w_dev,
                             int64_t n, float *grad_dev, double *loss);
/* Train on n device samples with log-weights ln w = lnLmargT + ln p - ln q. */
ile_status ile_prop_train_dev(ile_prop *p, const double *x_dev, int64_t ld,
                              const double *lnw_dev, int64_t n,
                              const ile_prop_train_opts *opts, double *final_loss);
/* ln q of device samples; with mix_ctx and eps > 0 the density of the
 * defensive mixture (1 - eps) q_net + eps q_hist (the context's histograms,
 * which must share the proposal's stream). */
ile_status ile_prop_logpdf_dev(ile_prop *p, const ile_ctx *mix_ctx, double eps,
                               const double *x_dev, int64_t ld, int64_t n, double *ln_q_dev);
/* Draw samples first .. first+n-1 of stream `seed` into x_dev[7][ld], with
 * ln p (may be NULL) and ln q of the (mixture) proposal. */
ile_status ile_prop_sample_dev(ile_prop *p, const ile_ctx *mix_ctx, double eps, uint64_t seed,
                               int64_t first, int64_t n, double *x_dev, int64_t ld,
                               double *ln_p_dev, double *ln_q_dev);
ile_status ile_prop_sync(ile_prop *p);
/* Device time in ms of the last training or draw (HIP events). */
double ile_prop_last_ms(ile_prop *p);
void ile_prop_destroy(ile_prop *p);
const char *ile_prop_last_error(const ile_prop *p);

/* ------------------------------------------------------ batched form
 * Many intrinsic points (Sec. III.B: each ILE instance loops over many
 * points to amortize its startup), each with its own detectors, modes,
 * window length and Q/U/V, evaluated together: one prior draw, one window
 * and ordering pass and one counting sort for all points, one persistent
 * contraction kernel draining a (point, tile) queue, and one per-point
 * reduction -- captured once in a HIP graph and replayed.  Point p draws
 * from the Philox stream of key seed + p (the stream of ile_draw_prior_dev).
 * Tuning (threads per workgroup, persistent workgroups per CU, queue order)
 * is set by hand or by ile_batch_autotune, which times the candidates and
 * caches the winner in a text file keyed by device, precision and the
 * points' shapes.  Defaults: matrix cores, 2 workgroups per CU, queue by
 * cost.  Default tuning: FP64 and FP32 on the phased matrix-core engine in
 * 512-thread workgroups, two per compute unit; BF16 on the pipelined engine
 * at 128 positions per block. */
typedef struct ile_batch ile_batch;

typedef struct {
    ile_precision precision;  /* bulk contraction precision of every point   */
    int32_t device;
    void *stream;             /* hipStream_t, or NULL for a new one          */
} ile_batch_config;

typedef struct {
    int32_t threads;          /* engine 1 for FP64/FP32: workgroup size, 256
                                 or 512; engines 2 and 0 (and 1 for BF16):
                                 positions per block, 256 or 512, 128 or 192
                                 with the matrix cores (BF16: 128 .. 256)    */
    int32_t wgs_per_cu;       /* persistent workgroups per compute unit, 1..4 */
    int32_t order;            /* 0: queue by decreasing cost, 1: point order  */
    int32_t engine;           /* 1 matrix cores (phased for FP64/FP32,
                                 pipelined for BF16), 2 matrix cores
                                 pipelined, 0 vector FMA (not for BF16)      */
} ile_batch_tuning;

ile_status ile_batch_create(const ile_batch_config *cfg, ile_batch **out);
/* Add one point: cfg describes it exactly as for ile_create (its precision,
 * device and stream fields are ignored), then Q/U/V/dets as ile_set_data.
 * The data are validated and copied; *id_out receives the point index. */
ile_status ile_batch_add_point(ile_batch *b, const ile_config *cfg, const double *Q,
                               int64_t n_q, double t0_s, const double *U,
                               const double *V, const ile_detector *dets,
                               int32_t *id_out);
/* Draw n_per_point prior samples per point, evaluate, reduce: results[p]
 * for every point p (host array of ile_batch_n_points entries). */
ile_status ile_batch_run(ile_batch *b, uint64_t seed, int64_t n_per_point, double d_min,
                         double d_max, ile_result *results);
/* The same graph over caller-supplied draws (the combined form: each point
 * drawn from its own proposal): device samples_dev[P][7][n_per_point]
 * (point p's SoA block at samples_dev + 7 n_per_point p), ln_p_dev and
 * ln_q_dev [P][n_per_point] (either may be NULL = 0); the per-point
 * reduction weighs each draw by ln L_margT + ln p - ln q.  The draws are
 * copied first, so the caller's buffers are free when this returns.
 * ILE_E_RANGE if a draw is outside a point's prior support or its window
 * leaves its Q, or if a ln p / ln q is NaN, ln q = -inf or ln p = +inf. */
ile_status ile_batch_run_dev(ile_batch *b, int64_t n_per_point, const double *samples_dev,
                             const double *ln_p_dev, const double *ln_q_dev,
                             ile_result *results);
/* Per-point ln L_margT of the last run into host out[offset of p + i]
 * (points concatenated, n_per_point each). */
ile_status ile_batch_lnL(ile_batch *b, double *out, int64_t n_total);
int32_t ile_batch_n_points(const ile_batch *b);
ile_status ile_batch_set_tuning(ile_batch *b, const ile_batch_tuning *t);
ile_status ile_batch_get_tuning(const ile_batch *b, ile_batch_tuning *t);
/* Time every candidate tuning on a run of n_per_point samples per point and
 * keep the fastest; cache_path (may be NULL) is read first and updated. */
ile_status ile_batch_autotune(ile_batch *b, int64_t n_per_point, const char *cache_path);
/* Device time in ms of the last run's graph (HIP events on its stream). */
double ile_batch_last_ms(const ile_batch *b);
void ile_batch_destroy(ile_batch *b);
const char *ile_batch_last_error(const ile_batch *b);

/* The context's stream (hipStream_t): the one its device calls are
 * ordered on, to share with a proposal. */
ile_status ile_get_stream(const ile_ctx *ctx, void **stream_out);

/* Wait for the context's stream; report a sticky device-side error. */
ile_status ile_sync(ile_ctx *ctx);

typedef enum {
    ILE_OPT_SORT = 0,    /* 1: order samples by window position before the
                            contraction (default), 0: keep input order */
    ILE_OPT_ENGINE = 1,  /* contraction engine: 1 = matrix cores (default):
                            for FP64 and FP32 the phased form, in which
                            every wave of a tile computes its share of the
                            windowed products and then time-marginalizes
                            its share of the samples; for BF16 the
                            pipelined form.  2 = matrix cores, pipelined:
                            producer waves compute the products while
                            consumer waves marginalize the previous block.
                            0 = vector FMA (a block width of 128 or 192
                            becomes 256) */
    ILE_OPT_THREADS = 2, /* pipelined and vector engines: positions per
                            block, 256 or 512, or 128 or 192 with the
                            matrix cores (workgroups of twice as many
                            threads: producers + consumers); default 128
                            for FP64 and BF16, 256 for FP32 */
    ILE_OPT_HARVEST_ROWS = 3, /* most draws whose per-bin series
                            ile_harvest_dev holds at once (>= 1; 0 restores
                            the default of 2 GiB of series) */
    ILE_OPT_LDS_KB = 4   /* phased engine: LDS per workgroup in KiB for its
                            coefficient and product blocks (0 .. 160; 0
                            restores the default of 78, two workgroups per
                            compute unit).  A larger budget gives longer
                            time chunks and fewer workgroups per unit; a
                            budget too small for a 32-position block makes
                            the evaluation fail with ILE_E_UNSUPPORTED */
} ile_option;
ile_status ile_set_option(ile_ctx *ctx, ile_option opt, int64_t value);

/* Average duration in ms of the last launch of the contraction kernel
 * (HIP events around it on the context's stream); 0 if none. */
double ile_last_kernel_ms(const ile_ctx *ctx);

void ile_destroy(ile_ctx *ctx);
const char *ile_last_error(const ile_ctx *ctx);
const char *ile_status_string(ile_status s);

#ifdef __cplusplus
}
#endif
#endif /* ILE_H */
