// ile_prop_api.cpp -- host side of the learned proposal (ile_prop_*): device
// state, argument checks, training loop and the draws of the defensive
// mixture.  Conventions as for the rest of the C ABI (include/ile.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ile.h"
#include "ile_internal.h"

struct ile_prop {
    ile_prop_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int grid = 256;              // persistent inference workgroups (one per CU)
    std::string err;
    ile_mdn_dev M{};
    ile_mdn_tr tr{};             // host copy of the device transform
    // training scratch
    void *part = nullptr, *idx = nullptr, *z = nullptr, *w = nullptr, *cdf = nullptr,
         *stats = nullptr, *loss = nullptr, *ws = nullptr;
    size_t part_b = 0, idx_b = 0, z_b = 0, w_b = 0, cdf_b = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double last_ms = 0.0;
};

namespace {

ile_status pfail(ile_prop *p, ile_status s, const char *fmt, ...)
{
    if (p) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        p->err = buf;
    }
    return s;
}

#define PHIP(p, expr)                                                            \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            return pfail((p), e_ == hipErrorOutOfMemory ? ILE_E_NOMEM : ILE_E_DEVICE, \
                         "%s: %s", #expr, hipGetErrorString(e_));                \
    } while (0)

ile_status grow(ile_prop *p, void *&buf, size_t &have, size_t bytes)
{
    if (have >= bytes && buf) return ILE_OK;
    if (buf) {
        PHIP(p, hipStreamSynchronize(p->stream));
        (void)hipFree(buf);
        buf = nullptr;
        have = 0;
    }
    bytes = std::max<size_t>(bytes, 256);
    PHIP(p, hipMalloc(&buf, bytes));
    have = bytes;
    return ILE_OK;
}

// splitmix64 (Steele, Lea, Flood 2014) for the initial weights
uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double unif(uint64_t &s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// Glorot-uniform weights (W3 at half gain), zero biases except the output
// layer: mixture means spread over [-2, 2], scales near 1/2.
std::vector<float> initial_params(uint64_t seed)
{
    std::vector<float> P(ILE_MDN_NPARAM, 0.f);
    uint64_t s = seed ^ 0x6D646E5F696E6974ull;
    auto fill = [&](int off, int n, int fan_in, int fan_out, double gain) {
        const double a = gain * std::sqrt(6.0 / (fan_in + fan_out));
        for (int j = 0; j < n; j++) P[off + j] = (float)(a * (2.0 * unif(s) - 1.0));
    };
    fill(ILE_MDN_OFF_W1, ILE_MDN_H * ILE_MDN_D, ILE_MDN_D, ILE_MDN_H, 1.0);
    fill(ILE_MDN_OFF_W2, ILE_MDN_H * ILE_MDN_H, ILE_MDN_H, ILE_MDN_H, 1.0);
    fill(ILE_MDN_OFF_W3, ILE_MDN_O * ILE_MDN_H, ILE_MDN_H, ILE_MDN_O, 0.5);
    for (int d = 0; d < ILE_MDN_D; d++)
        for (int c = 0; c < ILE_MDN_C; c++) {
            P[ILE_MDN_OFF_B3 + 48 * d + 16 + c] = (float)(-2.0 + 4.0 * c / (ILE_MDN_C - 1));
            P[ILE_MDN_OFF_B3 + 48 * d + 32 + c] = (float)std::log(std::expm1(0.5));
        }
    for (int j = 0; j < ILE_MDN_NPARAM; j++)
        if (!ile_mdn_trainable(j)) P[j] = 0.f;
    return P;
}

ile_status upload_tr(ile_prop *p)
{
    PHIP(p, hipMemcpyAsync(p->M.tr, &p->tr, sizeof(ile_mdn_tr), hipMemcpyHostToDevice,
                           p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    return ILE_OK;
}

ile_status download_tr(ile_prop *p)
{
    PHIP(p, hipStreamSynchronize(p->stream));
    PHIP(p, hipMemcpy(&p->tr, p->M.tr, sizeof(ile_mdn_tr), hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status mix_of(ile_prop *p, const ile_ctx *ctx, double eps, ile_mdn_mix &mix)
{
    mix = ile_mdn_mix{0, nullptr, nullptr, 0.0};
    if (!(eps >= 0.0 && eps < 1.0)) return pfail(p, ILE_E_ARG, "eps must be in [0, 1)");
    if (eps == 0.0) return ILE_OK;
    if (!ctx) return pfail(p, ILE_E_ARG, "eps > 0 needs a context with histograms");
    if (ile_ctx_stream(ctx) != p->stream)
        return pfail(p, ILE_E_ARG, "the context and the proposal must share a stream");
    const double *P = nullptr, *C = nullptr;
    const int nb = ile_ctx_hist(ctx, &P, &C);
    if (nb <= 0) return pfail(p, ILE_E_STATE, "the context has no histogram proposal yet");
    mix = ile_mdn_mix{nb, P, C, eps};
    return ILE_OK;
}

ile_status check_x(ile_prop *p, const double *x, int64_t ld, int64_t n)
{
    if (n < 0 || (n > 0 && !x) || ld < n) return pfail(p, ILE_E_ARG, "bad sample array");
    if (n > ((int64_t)1 << 31) - 64) return pfail(p, ILE_E_ARG, "too many samples");
    return ILE_OK;
}

}  // namespace

const ile_mdn_dev &ile_prop_dev(const ile_prop *p) { return p->M; }
hipStream_t ile_prop_stream(const ile_prop *p) { return p->stream; }
int ile_prop_grid(const ile_prop *p) { return p->grid; }

extern "C" {

ile_status ile_prop_create(const ile_prop_config *cfg, ile_prop **out)
{
    if (!cfg || !out) return ILE_E_ARG;
    *out = nullptr;
    if (!(cfg->d_min_mpc > 0) || !(cfg->d_max_mpc > cfg->d_min_mpc) ||
        !std::isfinite(cfg->d_max_mpc) || !(cfg->t_ref_max_s > 0) ||
        !std::isfinite(cfg->t_ref_max_s))
        return ILE_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ILE_E_DEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return ILE_E_ARG;
    ile_prop *p = new (std::nothrow) ile_prop;
    if (!p) return ILE_E_NOMEM;
    p->cfg = *cfg;
    auto bail = [&](ile_status s) {
        ile_prop_destroy(p);
        return s;
    };
    if (hipSetDevice(cfg->device) != hipSuccess) return bail(ILE_E_DEVICE);
    if (cfg->stream) {
        p->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreate(&p->stream) != hipSuccess)
            return bail(ILE_E_DEVICE);
        p->own_stream = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return bail(ILE_E_DEVICE);
    p->grid = std::max(1, prop.multiProcessorCount);
    const size_t NP = ILE_MDN_NPARAM;
    bool ok = hipMalloc((void **)&p->M.theta, NP * 4) == hipSuccess &&
              hipMalloc((void **)&p->M.m, NP * 4) == hipSuccess &&
              hipMalloc((void **)&p->M.v, NP * 4) == hipSuccess &&
              hipMalloc((void **)&p->M.W2b, ILE_MDN_H * ILE_MDN_H * 2) == hipSuccess &&
              hipMalloc((void **)&p->M.W2t, ILE_MDN_H * ILE_MDN_H * 2) == hipSuccess &&
              hipMalloc((void **)&p->M.W3b, ILE_MDN_O * ILE_MDN_H * 2) == hipSuccess &&
              hipMalloc((void **)&p->M.W3t, ILE_MDN_H * ILE_MDN_W3T_LD * 2) == hipSuccess &&
              hipMalloc((void **)&p->M.tr, sizeof(ile_mdn_tr)) == hipSuccess &&
              hipMalloc(&p->stats, 4 * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->ws, ile_mdn_fit_ws_doubles() * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->loss, sizeof(double)) == hipSuccess &&
              hipEventCreate(&p->ev[0]) == hipSuccess && hipEventCreate(&p->ev[1]) == hipSuccess;
    if (!ok) return bail(ILE_E_NOMEM);
    p->tr = ile_mdn_tr{};
    for (int d = 0; d < 7; d++) p->tr.scale[d] = 1.0;
    p->tr.d_min = cfg->d_min_mpc;
    p->tr.d_max = cfg->d_max_mpc;
    p->tr.t_ref_max = cfg->t_ref_max_s;
    p->tr.sigma_floor = cfg->sigma_floor > 0 ? cfg->sigma_floor : 1e-3;
    p->tr.sigma_scale = cfg->sigma_scale > 0 ? cfg->sigma_scale : 1.0;
    std::vector<float> P0 = initial_params(cfg->seed);
    // the zero tail of the transposed W3 copy (outputs 336..383) is never written again
    if (hipMemsetAsync(p->M.W3t, 0, ILE_MDN_H * ILE_MDN_W3T_LD * 2, p->stream) != hipSuccess ||
        hipMemsetAsync(p->M.m, 0, NP * 4, p->stream) != hipSuccess ||
        hipMemsetAsync(p->M.v, 0, NP * 4, p->stream) != hipSuccess ||
        hipMemcpyAsync(p->M.theta, P0.data(), NP * 4, hipMemcpyHostToDevice, p->stream) !=
            hipSuccess ||
        ile_launch_mdn_cast(p->M, p->stream) != hipSuccess || upload_tr(p) != ILE_OK)
        return bail(ILE_E_DEVICE);
    *out = p;
    return ILE_OK;
}

ile_status ile_prop_set_params(ile_prop *p, const float *params)
{
    if (!p) return ILE_E_ARG;
    if (!params) return pfail(p, ILE_E_ARG, "null pointer");
    std::vector<float> P(params, params + ILE_MDN_NPARAM);
    for (int j = 0; j < ILE_MDN_NPARAM; j++) {
        if (!std::isfinite(P[j])) return pfail(p, ILE_E_NUMERIC, "parameter %d not finite", j);
        if (!ile_mdn_trainable(j)) P[j] = 0.f;
    }
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, hipMemcpyAsync(p->M.theta, P.data(), ILE_MDN_NPARAM * 4, hipMemcpyHostToDevice,
                           p->stream));
    PHIP(p, hipMemsetAsync(p->M.m, 0, ILE_MDN_NPARAM * 4, p->stream));
    PHIP(p, hipMemsetAsync(p->M.v, 0, ILE_MDN_NPARAM * 4, p->stream));
    PHIP(p, ile_launch_mdn_cast(p->M, p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    return ILE_OK;
}

ile_status ile_prop_get_params(ile_prop *p, float *params)
{
    if (!p) return ILE_E_ARG;
    if (!params) return pfail(p, ILE_E_ARG, "null pointer");
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, hipStreamSynchronize(p->stream));
    PHIP(p, hipMemcpy(params, p->M.theta, ILE_MDN_NPARAM * 4, hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_prop_set_transform(ile_prop *p, const double origin[3], const double mean[7],
                                  const double scale[7])
{
    if (!p) return ILE_E_ARG;
    if (!origin || !mean || !scale) return pfail(p, ILE_E_ARG, "null pointer");
    for (int d = 0; d < 7; d++)
        if (!std::isfinite(mean[d]) || !(scale[d] > 0) || !std::isfinite(scale[d]))
            return pfail(p, ILE_E_ARG, "bad mean/scale of dimension %d", d);
    for (int j = 0; j < 3; j++)
        if (!std::isfinite(origin[j])) return pfail(p, ILE_E_ARG, "bad origin %d", j);
    PHIP(p, hipSetDevice(p->cfg.device));
    memcpy(p->tr.origin, origin, sizeof(p->tr.origin));
    memcpy(p->tr.mean, mean, sizeof(p->tr.mean));
    memcpy(p->tr.scale, scale, sizeof(p->tr.scale));
    return upload_tr(p);
}

ile_status ile_prop_get_transform(ile_prop *p, double origin[3], double mean[7], double scale[7])
{
    if (!p) return ILE_E_ARG;
    if (!origin || !mean || !scale) return pfail(p, ILE_E_ARG, "null pointer");
    PHIP(p, hipSetDevice(p->cfg.device));
    ile_status s = download_tr(p);
    if (s) return s;
    memcpy(origin, p->tr.origin, sizeof(p->tr.origin));
    memcpy(mean, p->tr.mean, sizeof(p->tr.mean));
    memcpy(scale, p->tr.scale, sizeof(p->tr.scale));
    return ILE_OK;
}

ile_status ile_prop_set_sigma_scale(ile_prop *p, double kappa)
{
    if (!p) return ILE_E_ARG;
    if (!(kappa > 0) || !std::isfinite(kappa)) return pfail(p, ILE_E_ARG, "sigma scale must be > 0");
    PHIP(p, hipSetDevice(p->cfg.device));
    ile_status s = download_tr(p);   // keep what a fit left on the device
    if (s) return s;
    p->tr.sigma_scale = kappa;
    return upload_tr(p);
}

ile_status ile_prop_fit_transform_dev(ile_prop *p, const double *x, int64_t ld, const double *lnw,
                                      int64_t n, double ess_frac)
{
    if (!p) return ILE_E_ARG;
    ile_status s = check_x(p, x, ld, n);
    if (s) return s;
    if (n <= 0 || !lnw) return pfail(p, ILE_E_ARG, "need n > 0 samples and their ln w");
    if (!(ess_frac > 0)) ess_frac = 0.01;
    if (ess_frac > 1) return pfail(p, ILE_E_ARG, "ess_frac must be in (0, 1]");
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, ile_launch_mdn_fit(x, ld, lnw, n, ess_frac, p->M.tr, (double *)p->stats,
                               (double *)p->ws, true, p->stream));
    return download_tr(p);
}

ile_status ile_prop_grad_dev(ile_prop *p, const double *x, int64_t ld, const double *w,
                             int64_t n, float *grad, double *loss)
{
    if (!p) return ILE_E_ARG;
    ile_status s = check_x(p, x, ld, n);
    if (s) return s;
    if (n <= 0 || n > (1 << 20)) return pfail(p, ILE_E_ARG, "batch must be in [1, 2^20]");
    PHIP(p, hipSetDevice(p->cfg.device));
    const int64_t nblk = (n + ILE_MDN_TILE - 1) / ILE_MDN_TILE;
    if ((s = grow(p, p->z, p->z_b, (size_t)n * 7 * sizeof(float)))) return s;
    if ((s = grow(p, p->w, p->w_b, (size_t)n * sizeof(double)))) return s;
    if ((s = grow(p, p->part, p->part_b, (size_t)nblk * ILE_MDN_NPART * sizeof(float)))) return s;
    PHIP(p, ile_launch_mdn_prepare_w(p->M.tr, x, ld, w, n, (float *)p->z, (double *)p->w,
                                     p->stream));
    PHIP(p, ile_launch_mdn_grad(p->M, (const float *)p->z, n, nullptr, (const double *)p->w,
                                (int)n, (float *)p->part, p->stream));
    PHIP(p, ile_launch_mdn_update(p->M, (const float *)p->part, (int)nblk, grad,
                                  (double *)p->loss, false, 0, 0.0, p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    if (loss) PHIP(p, hipMemcpy(loss, p->loss, sizeof(double), hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_prop_train_dev(ile_prop *p, const double *x, int64_t ld, const double *lnw,
                              int64_t n, const ile_prop_train_opts *o, double *final_loss)
{
    if (!p) return ILE_E_ARG;
    ile_status s = check_x(p, x, ld, n);
    if (s) return s;
    if (n <= 0 || !lnw) return pfail(p, ILE_E_ARG, "need n > 0 samples and their ln w");
    ile_prop_train_opts d{};
    if (o) d = *o;
    const int steps = d.steps > 0 ? d.steps : 1000;
    const int batch = d.batch > 0 ? d.batch : 4096;
    const double lr = d.lr > 0 ? d.lr : 1e-3;
    const double ess_frac = d.ess_frac > 0 ? d.ess_frac : 0.01;
    if (batch > (1 << 20) || ess_frac > 1 || (int64_t)batch * steps > ((int64_t)1 << 28))
        return pfail(p, ILE_E_ARG, "batch, steps or ess_frac out of range");
    PHIP(p, hipSetDevice(p->cfg.device));
    const int nblk = (batch + ILE_MDN_TILE - 1) / ILE_MDN_TILE;
    if ((s = grow(p, p->z, p->z_b, (size_t)n * 7 * sizeof(float)))) return s;
    if ((s = grow(p, p->w, p->w_b, (size_t)n * sizeof(double)))) return s;
    if ((s = grow(p, p->cdf, p->cdf_b, (size_t)n * sizeof(double)))) return s;
    if ((s = grow(p, p->idx, p->idx_b, (size_t)batch * steps * sizeof(int32_t)))) return s;
    if ((s = grow(p, p->part, p->part_b, (size_t)nblk * ILE_MDN_NPART * sizeof(float)))) return s;
    PHIP(p, ile_launch_mdn_fit(x, ld, lnw, n, ess_frac, p->M.tr, (double *)p->stats,
                               (double *)p->ws, d.fit_transform != 0, p->stream));
    PHIP(p, ile_launch_mdn_prepare(p->M.tr, x, ld, lnw, n, (const double *)p->stats,
                                   (float *)p->z, (double *)p->w, p->stream));
    PHIP(p, ile_launch_mdn_cdf((const double *)p->w, n, (double *)p->cdf, (double *)p->ws,
                               p->stream));
    PHIP(p, hipEventRecord(p->ev[0], p->stream));
    PHIP(p, ile_launch_mdn_draw_idx(d.seed, (int64_t)batch * steps, (const double *)p->cdf, n,
                                    (int32_t *)p->idx, p->stream));
    for (int t = 0; t < steps; t++) {
        PHIP(p, ile_launch_mdn_grad(p->M, (const float *)p->z, n,
                                    (const int32_t *)p->idx + (size_t)t * batch, nullptr, batch,
                                    (float *)p->part, p->stream));
        PHIP(p, ile_launch_mdn_update(p->M, (const float *)p->part, nblk, nullptr,
                                      t == steps - 1 ? (double *)p->loss : nullptr, true, t + 1,
                                      lr, p->stream));
    }
    PHIP(p, hipEventRecord(p->ev[1], p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    float ms = 0.f;
    PHIP(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->last_ms = ms;
    if (d.fit_transform && (s = download_tr(p))) return s;
    if (final_loss) PHIP(p, hipMemcpy(final_loss, p->loss, sizeof(double), hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_prop_logpdf_dev(ile_prop *p, const ile_ctx *mix_ctx, double eps, const double *x,
                               int64_t ld, int64_t n, double *ln_q)
{
    if (!p) return ILE_E_ARG;
    ile_status s = check_x(p, x, ld, n);
    if (s) return s;
    if (n > 0 && !ln_q) return pfail(p, ILE_E_ARG, "null output");
    ile_mdn_mix mix;
    if ((s = mix_of(p, mix_ctx, eps, mix))) return s;
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, ile_launch_mdn_logpdf(p->M, mix, x, ld, n, ln_q, p->grid, p->stream));
    return ILE_OK;
}

ile_status ile_prop_sample_dev(ile_prop *p, const ile_ctx *mix_ctx, double eps, uint64_t seed,
                               int64_t first, int64_t n, double *x, int64_t ld, double *ln_p,
                               double *ln_q)
{
    if (!p) return ILE_E_ARG;
    ile_status s = check_x(p, x, ld, n);
    if (s) return s;
    if (first < 0 || (n > 0 && !ln_q)) return pfail(p, ILE_E_ARG, "bad first or null ln_q");
    ile_mdn_mix mix;
    if ((s = mix_of(p, mix_ctx, eps, mix))) return s;
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, hipEventRecord(p->ev[0], p->stream));
    PHIP(p, ile_launch_mdn_sample(p->M, mix, seed, first, n, x, ld, ln_p, ln_q, p->grid,
                                  p->stream));
    PHIP(p, hipEventRecord(p->ev[1], p->stream));
    return ILE_OK;
}

ile_status ile_prop_sync(ile_prop *p)
{
    if (!p) return ILE_E_ARG;
    PHIP(p, hipSetDevice(p->cfg.device));
    PHIP(p, hipStreamSynchronize(p->stream));
    return ILE_OK;
}

double ile_prop_last_ms(ile_prop *p)
{
    if (!p) return 0.0;
    float ms = 0.f;
    if (hipEventSynchronize(p->ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, p->ev[0], p->ev[1]) == hipSuccess)
        return ms;
    return p->last_ms;
}

void ile_prop_destroy(ile_prop *p)
{
    if (!p) return;
    (void)hipSetDevice(p->cfg.device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    void *bufs[] = {p->M.theta, p->M.m, p->M.v, p->M.W2b, p->M.W3b, p->M.W2t, p->M.W3t, p->M.tr,
                    p->part, p->idx, p->z, p->w, p->cdf, p->stats, p->loss, p->ws};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

const char *ile_prop_last_error(const ile_prop *p) { return p ? p->err.c_str() : "null proposal"; }

}  // extern "C"
