/*
 * mdn_oracle.h -- plain FP64 CPU oracle of the learned proposal.
 *
 * TEST INFRASTRUCTURE ONLY (like ile_oracle.h): only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark use it; it shares no
 * source with the HIP path.
 *
 * The paper adapts its sampling distribution with one-dimensional
 * histograms (Sec. II.A, Sec. III.C); a learned proposal is not part of it.
 * This is the model the library trains in its place of a richer adaptive
 * density: a masked autoregressive (MADE) network whose outputs are, for
 * each of the 7 transformed extrinsic parameters, a 16-component Gaussian
 * mixture conditioned on the parameters before it.
 *
 * Model (shared definition with the library; the flat parameter layout is
 * part of the C ABI):
 *   inputs  z~[7]  (transformed parameters, order of the sample vector)
 *   a1 = (W1 . M1) z~ + b1,  h1 = tanh(a1)            W1 [128][7]
 *   a2 = (W2 . M2) h1 + b2,  h2 = tanh(a2)            W2 [128][128]
 *   o  = (W3 . M3) h2 + b3                             W3 [336][128]
 *   params = W1 | b1 | W2 | b2 | W3 | b3  (60880 values, row-major)
 *   hidden degree m(k) = k mod 6; masks
 *     M1[k][i] = (i <= m(k)), M2[k'][k] = (m(k) <= m(k')),
 *     M3[o][k] = (m(k) < o / 48)
 *   dimension d uses o[48d + c] (mixture logit), o[48d + 16 + c] (mean),
 *   o[48d + 32 + c] (scale pre-activation rho), c = 0..15;
 *   sigma = kappa (sigma_floor + softplus(rho)), kappa = sigma_scale: a
 *   widening of every component for drawing and evaluating; the training
 *   loss is that of the kappa = 1 model.
 *   ln q(z~) = sum_d log sum_c softmax(logits)_c N(z~_d; mean_c, sigma_c)
 *
 * Transform x -> z~ (x = ra, dec, psi, phi, cos iota, D, t_ref):
 *   u = frac((x - origin)/P + 1/2) for the periodic ra (P = 2 pi),
 *   psi (P = pi), phi (P = 2 pi); u = (sin dec + 1)/2; u = (cos iota + 1)/2;
 *   u = (D - d_min)/(d_max - d_min); u = (t_ref + t_max)/(2 t_max);
 *   z = log(u/(1-u)), z~ = (z - mean)/scale.
 *   ln q(x) = ln q(z~) + sum_d ln |dz~_d/dx_d|; -inf if any u is 0 or 1.
 */
#ifndef MDN_ORACLE_H
#define MDN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MDN_D 7
#define ORC_MDN_H 128
#define ORC_MDN_C 16
#define ORC_MDN_O (ORC_MDN_D * 3 * ORC_MDN_C)
#define ORC_MDN_OFF_W1 0
#define ORC_MDN_OFF_B1 (ORC_MDN_OFF_W1 + ORC_MDN_H * ORC_MDN_D)
#define ORC_MDN_OFF_W2 (ORC_MDN_OFF_B1 + ORC_MDN_H)
#define ORC_MDN_OFF_B2 (ORC_MDN_OFF_W2 + ORC_MDN_H * ORC_MDN_H)
#define ORC_MDN_OFF_W3 (ORC_MDN_OFF_B2 + ORC_MDN_H)
#define ORC_MDN_OFF_B3 (ORC_MDN_OFF_W3 + ORC_MDN_O * ORC_MDN_H)
#define ORC_MDN_NPARAM (ORC_MDN_OFF_B3 + ORC_MDN_O)

typedef struct {
    double origin[3];     /* ra, psi, phi origins [rad] */
    double mean[7], scale[7];
    double d_min, d_max, t_ref_max;
    double sigma_floor;
    double sigma_scale;   /* kappa of the density (training uses 1) */
} orc_mdn_transform;

/* Mask value of parameter index j (1 = trainable, 0 = held at zero). */
int orc_mdn_mask(int64_t j);

/* x -> z~ for one sample (x[7]); returns ln |dz~/dx| summed over the 7
 * dimensions, or -INFINITY (z~ then undefined) if a u falls outside (0,1). */
double orc_mdn_to_z(const orc_mdn_transform *tr, const double x[7], double z[7]);

/* ln q(z~) of one transformed sample and, if lnq_dim is not NULL, its 7
 * per-dimension terms. */
double orc_mdn_lnq_z(const double *params, const orc_mdn_transform *tr,
                     const double z[7], double *lnq_dim);

/* ln q(x) of n samples x[7][ld] (SoA). */
void orc_mdn_logpdf(const double *params, const orc_mdn_transform *tr,
                    const double *x, int64_t ld, int64_t n, double *lnq);

/* z~ (z_out[n][7]) and the 336 network outputs (o_out[n][336]) of n samples
 * x[7][ld]; for each dimension d the outputs 48d.. give the conditional
 * mixture given z~_0..z~_{d-1}. */
void orc_mdn_outputs(const double *params, const orc_mdn_transform *tr, const double *x,
                     int64_t ld, int64_t n, double *z_out, double *o_out);

/* Weighted negative log-likelihood in z~ space of the kappa = 1 model
 * (tr->sigma_scale is not used),
 *   loss = -sum_i w_i ln q(z~_i) / sum_i w_i     (w = NULL: all 1),
 * and its gradient with respect to every parameter (masked entries 0), by
 * hand-written back-propagation. */
void orc_mdn_loss_grad(const double *params, const orc_mdn_transform *tr,
                       const double *x, int64_t ld, int64_t n, const double *w,
                       double *loss, double *grad);

/* Tempering of training weights w = exp(beta (lnw - max)) over the finite
 * lnw: beta = 1 if the Kish effective size (sum w)^2 / sum w^2 is at least
 * max(1, ess_frac * count), else the bisection of [0, 1] (30 halvings,
 * keeping the lower end) for the largest beta whose effective size reaches
 * that target.  Returns beta; *max_out (may be NULL) = max lnw. */
double orc_mdn_tempering(const double *lnw, int64_t n, double ess_frac, double *max_out);

/* Transform fit from weighted samples with the tempered weights above:
 * origins = weighted circular means; mean/scale = weighted mean and
 * standard deviation of z (scale floored at 1e-3); non-finite ln w weigh
 * 0.  Moment sums in index order (long double). */
void orc_mdn_fit_transform(const double *x, int64_t ld, const double *lnw,
                           int64_t n, double ess_frac, orc_mdn_transform *tr);

#ifdef __cplusplus
}
#endif
#endif
