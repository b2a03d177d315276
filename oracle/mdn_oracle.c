/*
 * mdn_oracle.c -- plain FP64 CPU oracle of the learned proposal (model and
 * transform defined in mdn_oracle.h).  TEST INFRASTRUCTURE ONLY.
 *
 * Written for checking, not speed: dense loops in the order of the
 * definitions, masks applied by multiplying each weight by its mask,
 * back-propagation by the chain rule one layer at a time.
 */
#include "mdn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

static const int PERIODIC_DIM[3] = {0, 2, 3};

static int hdeg(int k) { return k % 6; }

int orc_mdn_mask(int64_t j)
{
    if (j < 0 || j >= ORC_MDN_NPARAM) return 0;
    if (j >= ORC_MDN_OFF_W1 && j < ORC_MDN_OFF_B1) {
        int64_t r = j - ORC_MDN_OFF_W1;
        int k = (int)(r / ORC_MDN_D), i = (int)(r % ORC_MDN_D);
        return i <= hdeg(k);
    }
    if (j >= ORC_MDN_OFF_W2 && j < ORC_MDN_OFF_B2) {
        int64_t r = j - ORC_MDN_OFF_W2;
        int k2 = (int)(r / ORC_MDN_H), k1 = (int)(r % ORC_MDN_H);
        return hdeg(k1) <= hdeg(k2);
    }
    if (j >= ORC_MDN_OFF_W3 && j < ORC_MDN_OFF_B3) {
        int64_t r = j - ORC_MDN_OFF_W3;
        int o = (int)(r / ORC_MDN_H), k = (int)(r % ORC_MDN_H);
        return hdeg(k) < o / (3 * ORC_MDN_C);
    }
    return 1; /* biases */
}

static double softplus(double r) { return fmax(r, 0.0) + log1p(exp(-fabs(r))); }
static double sigmoid(double r) { return 1.0 / (1.0 + exp(-r)); }

/* u in (0,1) and du/dx of dimension d */
static void unit_of(const orc_mdn_transform *tr, int d, double x, double *u, double *dudx)
{
    switch (d) {
    case 0: {
        double y = (x - tr->origin[0]) / (2 * PI) + 0.5;
        *u = y - floor(y);
        *dudx = 1.0 / (2 * PI);
        break;
    }
    case 1:
        *u = (sin(x) + 1.0) / 2.0;
        *dudx = cos(x) / 2.0;
        break;
    case 2: {
        double y = (x - tr->origin[1]) / PI + 0.5;
        *u = y - floor(y);
        *dudx = 1.0 / PI;
        break;
    }
    case 3: {
        double y = (x - tr->origin[2]) / (2 * PI) + 0.5;
        *u = y - floor(y);
        *dudx = 1.0 / (2 * PI);
        break;
    }
    case 4:
        *u = (x + 1.0) / 2.0;
        *dudx = 0.5;
        break;
    case 5:
        *u = (x - tr->d_min) / (tr->d_max - tr->d_min);
        *dudx = 1.0 / (tr->d_max - tr->d_min);
        break;
    default:
        *u = (x + tr->t_ref_max) / (2.0 * tr->t_ref_max);
        *dudx = 1.0 / (2.0 * tr->t_ref_max);
        break;
    }
}

double orc_mdn_to_z(const orc_mdn_transform *tr, const double x[7], double z[7])
{
    double lj = 0.0;
    for (int d = 0; d < ORC_MDN_D; d++) {
        double u, dudx;
        unit_of(tr, d, x[d], &u, &dudx);
        if (!(u > 0.0 && u < 1.0)) return -INFINITY;
        double zz = log(u) - log1p(-u);
        z[d] = (zz - tr->mean[d]) / tr->scale[d];
        /* dz~/dx = (1/scale) (1/(u(1-u))) du/dx */
        lj += -log(tr->scale[d]) - log(u) - log1p(-u) + log(fabs(dudx));
    }
    return lj;
}

/* forward pass keeping the activations */
typedef struct {
    double h1[ORC_MDN_H], h2[ORC_MDN_H], o[ORC_MDN_O];
} fwd_state;

static void forward(const double *P, const double z[7], fwd_state *s)
{
    const double *W1 = P + ORC_MDN_OFF_W1, *b1 = P + ORC_MDN_OFF_B1;
    const double *W2 = P + ORC_MDN_OFF_W2, *b2 = P + ORC_MDN_OFF_B2;
    const double *W3 = P + ORC_MDN_OFF_W3, *b3 = P + ORC_MDN_OFF_B3;
    for (int k = 0; k < ORC_MDN_H; k++) {
        double a = b1[k];
        for (int i = 0; i < ORC_MDN_D; i++)
            a += W1[k * ORC_MDN_D + i] * (double)(i <= hdeg(k)) * z[i];
        s->h1[k] = tanh(a);
    }
    for (int k2 = 0; k2 < ORC_MDN_H; k2++) {
        double a = b2[k2];
        for (int k1 = 0; k1 < ORC_MDN_H; k1++)
            a += W2[k2 * ORC_MDN_H + k1] * (double)(hdeg(k1) <= hdeg(k2)) * s->h1[k1];
        s->h2[k2] = tanh(a);
    }
    for (int o = 0; o < ORC_MDN_O; o++) {
        double a = b3[o];
        for (int k = 0; k < ORC_MDN_H; k++)
            a += W3[o * ORC_MDN_H + k] * (double)(hdeg(k) < o / (3 * ORC_MDN_C)) * s->h2[k];
        s->o[o] = a;
    }
}

static double lse(const double *v, int n)
{
    double m = -INFINITY;
    for (int i = 0; i < n; i++) m = fmax(m, v[i]);
    if (m == -INFINITY) return m;
    double t = 0.0;
    for (int i = 0; i < n; i++) t += exp(v[i] - m);
    return m + log(t);
}

/* ln q_d of one dimension from its 48 outputs; if g is not NULL, writes
 * d ln q_d / d o for these 48 outputs. */
static double mixture_dim(const double *o, double zd, double sigma_floor, double kappa, double *g)
{
    const int C = ORC_MDN_C;
    const double *alpha = o, *mu = o + C, *rho = o + 2 * C;
    double la = lse(alpha, C);
    double l[ORC_MDN_C], sig[ORC_MDN_C], r[ORC_MDN_C];
    for (int c = 0; c < C; c++) {
        sig[c] = kappa * (sigma_floor + softplus(rho[c]));
        r[c] = (zd - mu[c]) / sig[c];
        l[c] = alpha[c] - la - 0.5 * r[c] * r[c] - log(sig[c]) - 0.5 * log(2 * PI);
    }
    double lq = lse(l, C);
    if (g) {
        for (int c = 0; c < C; c++) {
            double gam = exp(l[c] - lq);
            double pi = exp(alpha[c] - la);
            g[c] = gam - pi;
            g[C + c] = gam * r[c] / sig[c];
            g[2 * C + c] = gam * (r[c] * r[c] - 1.0) / sig[c] * sigmoid(rho[c]);
        }
    }
    return lq;
}

double orc_mdn_lnq_z(const double *params, const orc_mdn_transform *tr, const double z[7],
                     double *lnq_dim)
{
    fwd_state s;
    forward(params, z, &s);
    double tot = 0.0;
    for (int d = 0; d < ORC_MDN_D; d++) {
        double v = mixture_dim(s.o + 3 * ORC_MDN_C * d, z[d], tr->sigma_floor, tr->sigma_scale,
                               NULL);
        if (lnq_dim) lnq_dim[d] = v;
        tot += v;
    }
    return tot;
}

void orc_mdn_logpdf(const double *params, const orc_mdn_transform *tr, const double *x,
                    int64_t ld, int64_t n, double *lnq)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double xi[7], z[7];
        for (int d = 0; d < 7; d++) xi[d] = x[d * ld + i];
        double lj = orc_mdn_to_z(tr, xi, z);
        lnq[i] = (lj == -INFINITY) ? -INFINITY : orc_mdn_lnq_z(params, tr, z, NULL) + lj;
    }
}

void orc_mdn_loss_grad(const double *params, const orc_mdn_transform *tr, const double *x,
                       int64_t ld, int64_t n, const double *w, double *loss, double *grad)
{
    const double *W2 = params + ORC_MDN_OFF_W2, *W3 = params + ORC_MDN_OFF_W3;
    memset(grad, 0, sizeof(double) * ORC_MDN_NPARAM);
    /* samples outside the transform's domain (a u of 0 or 1) carry no weight */
    double wsum = 0.0, lsum = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double xi[7], z[7];
        for (int d = 0; d < 7; d++) xi[d] = x[d * ld + i];
        if (orc_mdn_to_z(tr, xi, z) != -INFINITY) wsum += w ? w[i] : 1.0;
    }
    for (int64_t i = 0; i < n; i++) {
        const double wi = (w ? w[i] : 1.0) / wsum;
        double xi[7], z[7];
        for (int d = 0; d < 7; d++) xi[d] = x[d * ld + i];
        if (orc_mdn_to_z(tr, xi, z) == -INFINITY) continue;
        fwd_state s;
        forward(params, z, &s);
        /* dL/do = -w_i d ln q / d o */
        double go[ORC_MDN_O];
        for (int d = 0; d < ORC_MDN_D; d++) {
            double *g = go + 3 * ORC_MDN_C * d;
            lsum -= wi * mixture_dim(s.o + 3 * ORC_MDN_C * d, z[d], tr->sigma_floor, 1.0, g);
            for (int c = 0; c < 3 * ORC_MDN_C; c++) g[c] *= -wi;
        }
        /* layer 3 */
        double gh2[ORC_MDN_H];
        for (int k = 0; k < ORC_MDN_H; k++) gh2[k] = 0.0;
        for (int o = 0; o < ORC_MDN_O; o++) {
            grad[ORC_MDN_OFF_B3 + o] += go[o];
            for (int k = 0; k < ORC_MDN_H; k++) {
                double m = (double)(hdeg(k) < o / (3 * ORC_MDN_C));
                grad[ORC_MDN_OFF_W3 + o * ORC_MDN_H + k] += m * go[o] * s.h2[k];
                gh2[k] += m * W3[o * ORC_MDN_H + k] * go[o];
            }
        }
        /* layer 2 */
        double ga2[ORC_MDN_H], gh1[ORC_MDN_H];
        for (int k = 0; k < ORC_MDN_H; k++) {
            ga2[k] = gh2[k] * (1.0 - s.h2[k] * s.h2[k]);
            gh1[k] = 0.0;
        }
        for (int k2 = 0; k2 < ORC_MDN_H; k2++) {
            grad[ORC_MDN_OFF_B2 + k2] += ga2[k2];
            for (int k1 = 0; k1 < ORC_MDN_H; k1++) {
                double m = (double)(hdeg(k1) <= hdeg(k2));
                grad[ORC_MDN_OFF_W2 + k2 * ORC_MDN_H + k1] += m * ga2[k2] * s.h1[k1];
                gh1[k1] += m * W2[k2 * ORC_MDN_H + k1] * ga2[k2];
            }
        }
        /* layer 1 */
        for (int k = 0; k < ORC_MDN_H; k++) {
            double ga1 = gh1[k] * (1.0 - s.h1[k] * s.h1[k]);
            grad[ORC_MDN_OFF_B1 + k] += ga1;
            for (int d = 0; d < ORC_MDN_D; d++)
                grad[ORC_MDN_OFF_W1 + k * ORC_MDN_D + d] += (double)(d <= hdeg(k)) * ga1 * z[d];
        }
    }
    *loss = lsum;
}

/* Kish effective size of the weights exp(beta (lnw - m)) over the finite lnw */
static double ess_at(const double *lnw, int64_t n, double m, double beta)
{
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(lnw[i])) continue;
        double e = exp(beta * (lnw[i] - m));
        s1 += e;
        s2 += e * e;
    }
    return s2 > 0 ? s1 * s1 / s2 : 0.0;
}

double orc_mdn_tempering(const double *lnw, int64_t n, double ess_frac, double *max_out)
{
    double mx = -INFINITY;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++)
        if (isfinite(lnw[i])) {
            mx = fmax(mx, lnw[i]);
            cnt++;
        }
    if (max_out) *max_out = mx;
    if (cnt == 0) return 1.0;
    const double target = fmax(1.0, ess_frac * (double)cnt);
    if (ess_at(lnw, n, mx, 1.0) >= target) return 1.0;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 30; it++) {
        double mid = 0.5 * (lo + hi);
        if (ess_at(lnw, n, mx, mid) >= target)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

void orc_mdn_fit_transform(const double *x, int64_t ld, const double *lnw, int64_t n,
                           double ess_frac, orc_mdn_transform *tr)
{
    /* samples whose ln w is not finite carry no weight */
    double mx;
    double beta = orc_mdn_tempering(lnw, n, ess_frac, &mx);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; i++) w[i] = isfinite(lnw[i]) ? exp(beta * (lnw[i] - mx)) : 0.0;
    /* circular means of the periodic dimensions */
    const double period[3] = {2 * PI, PI, 2 * PI};
    for (int j = 0; j < 3; j++) {
        long double sc = 0.0L, ss = 0.0L;
        const double *xd = x + PERIODIC_DIM[j] * ld;
        for (int64_t i = 0; i < n; i++) {
            double a = 2 * PI * xd[i] / period[j];
            sc += w[i] * cos(a);
            ss += w[i] * sin(a);
        }
        tr->origin[j] = atan2((double)ss, (double)sc) * period[j] / (2 * PI);
    }
    /* weighted moments of z = logit(u) */
    for (int d = 0; d < 7; d++) {
        tr->mean[d] = 0.0;
        tr->scale[d] = 1.0;
    }
    long double sw = 0.0L, s1[7] = {0}, s2[7] = {0};
    for (int64_t i = 0; i < n; i++) {
        int ok = 1;
        double zz[7];
        for (int d = 0; d < 7; d++) {
            double u, dudx;
            unit_of(tr, d, x[d * ld + i], &u, &dudx);
            if (!(u > 0.0 && u < 1.0)) ok = 0;
            else zz[d] = log(u) - log1p(-u);
        }
        if (!ok) continue;
        sw += w[i];
        for (int d = 0; d < 7; d++) {
            s1[d] += w[i] * zz[d];
            s2[d] += w[i] * zz[d] * zz[d];
        }
    }
    for (int d = 0; d < 7; d++) {
        double m = (double)(s1[d] / sw);
        double v = (double)(s2[d] / sw) - m * m;
        tr->mean[d] = m;
        tr->scale[d] = fmax(sqrt(fmax(v, 0.0)), 1e-3);
    }
    free(w);
}

void orc_mdn_outputs(const double *params, const orc_mdn_transform *tr, const double *x,
                     int64_t ld, int64_t n, double *z_out, double *o_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double xi[7], z[7];
        for (int d = 0; d < 7; d++) xi[d] = x[d * ld + i];
        if (orc_mdn_to_z(tr, xi, z) == -INFINITY)
            for (int d = 0; d < 7; d++) z[d] = NAN;
        fwd_state s;
        forward(params, z, &s);
        for (int d = 0; d < 7; d++) z_out[i * 7 + d] = z[d];
        for (int o = 0; o < ORC_MDN_O; o++) o_out[i * ORC_MDN_O + o] = s.o[o];
    }
}
