// ile_api.cpp -- host side of libile: contexts, argument and range checks,
// device buffers and the launch sequence of the hot path.  The C ABI is
// declared (with its conventions) in include/ile.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ile.h"
#include "ile_internal.h"

// Workspace of ile_integrate_dev_noalloc: a fixed array that every GPU the
// library runs on holds until the process ends.  Up to ILE_NOALLOC_MAX_N
// samples: 8 (lnL) + 4 n_det (window starts) + 8 (keys, order) + 8 (2 +
// 3 n_det + 2 n_lm) (the phased engine's per-sample terms) + 56 + 4 n_det
// (samples and window starts in tile order) bytes each, plus
// up to 2^21 + 1 bucket counts, their scan and the reduction partials.
// Host code never passes `scratch` itself to a kernel (in host code the name
// is a stand-in, not a device address): it takes the per-device address that
// hipGetSymbolAddress returned in ile_create.
constexpr size_t kNoAllocBytes =
    (size_t)ILE_NOALLOC_MAX_N *
        (8 + 4 * ILE_MAX_DET + 8 + 8 * (2 + 3 * ILE_MAX_DET + 2 * ILE_MAX_LM) + 56 + 4 * ILE_MAX_DET) +
    ((size_t)9 << 20);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ile_ctx;
// accessors used by the batched form (ile_batch_api.cpp)
const ile_geom &ile_ctx_geom(const ile_ctx *c);
const void *ile_ctx_Q(const ile_ctx *c);
const double *ile_ctx_U(const ile_ctx *c);
const double *ile_ctx_V(const ile_ctx *c);
ile_precision ile_ctx_precision(const ile_ctx *c);
const double *ile_ctx_uvt(const ile_ctx *c);

struct ile_ctx {
    ile_config cfg{};
    std::vector<ile_mode> modes;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    bool have_data = false;
    ile_geom g{};
    uint32_t n_buckets = 1;
    int sort = 1;
    ile_tune tune{16, 256, 1};
    int lds_max = 0;
    DevBuf Q, U, V;
    DevBuf uvt;                     // upper triangles of U_h and V_s (see ile_launch_contract)
    DevBuf smp, out, lnp, lnq, shifts, keys, perm, hist, scan_tmp, errflag,
        red_tmp, parts, res, series, terms, smp_s, sh_s;
    DevBuf hP, hC, bins, hist_tmp;  // adaptive proposal state and scratch
    int hist_nb = 0;
    DevBuf trx, trw;                // training set of the learned sampler
    DevBuf hv_w, hv_cdf, hv_ws, hv_part, hv_flag, hv_sel;   // harvest
    int64_t hv_rows = 0;            // draws per series chunk (0: 2 GiB of series)
    DevBuf fd_tmp, fd_flag, fd_in, fd_out;   // frequency-domain construction
    ile_geom rom_g{};               // surrogate form: physical modes' Y tables
    int rom_pow = 0;                // powers of lambda in the coefficients (0: not set)
    DevBuf rom_A, rom_Z;
    ile_learned_info learned{};
    std::vector<hipEvent_t> ev;   // pairs around contraction launches
    int n_ev_used = 0;
    double last_ms = 0.0;
    void *hpin = nullptr;   // pinned host words: the error flag, then the 6 result fields
};

namespace {

ile_status fail(ile_ctx *c, ile_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_TRY(ctx, expr)                                                       \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            return fail((ctx), e_ == hipErrorOutOfMemory ? ILE_E_NOMEM : ILE_E_DEVICE, \
                        "%s: %s", #expr, hipGetErrorString(e_));                 \
    } while (0)

ile_status ensure(ile_ctx *c, DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return ILE_OK;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, ILE_E_DEVICE, "sync: %s", hipGetErrorString(e));
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(c, ILE_E_NOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
    return ILE_OK;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Look up this device's copy of `scratch` once (device `dev` current).
hipError_t scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = (unsigned char *)p;
    return hipSuccess;
}

unsigned char *scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

// Wigner-d expansion of -2Y_lm (Goldberg et al. 1967) into the term table of
// the kernels: sqrt((2l+1)/4pi) sum_k (-1)^k sqrt((l+m)!(l-m)!(l+2)!(l-2)!)
// / ((l+m-k)!(l-2-k)! k! (k+2-m)!) cos^{2l+m-2-2k} sin^{2k+2-m}.
bool build_ylm_table(ile_geom &g, const std::vector<ile_mode> &modes)
{
    int nt = 0;
    for (size_t a = 0; a < modes.size(); a++) {
        int l = modes[a].l, m = modes[a].m;
        int kmin = std::max(0, m - 2), kmax = std::min(l + m, l - 2);
        g.mode_m[a] = m;
        g.mode_first[a] = nt;
        g.mode_nterm[a] = 0;
        double norm = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi)) *
                      std::sqrt(fact(l + m) * fact(l - m) * fact(l + 2) * fact(l - 2));
        for (int k = kmin; k <= kmax; k++) {
            if (nt >= ILE_MAX_TERMS) return false;
            double a_k = norm / (fact(l + m - k) * fact(l - 2 - k) * fact(k) * fact(k + 2 - m));
            g.term_a[nt] = (k % 2 == 0) ? a_k : -a_k;
            g.term_pw[nt] = (2 * l + m - 2 - 2 * k) | (2 * k + 2 - m) << 8;
            nt++;
            g.mode_nterm[a]++;
        }
        g.n_pw = std::max(g.n_pw, 2 * l + 1);
        g.m_max = std::max(g.m_max, std::abs(m));
    }
    return true;
}

void detector_frame(const ile_detector &d, double R, double r[3], double D[9])
{
    const double lat = d.lat_deg * kPi / 180.0, lon = d.lon_deg * kPi / 180.0;
    const double az = d.xarm_az_deg * kPi / 180.0;
    const double e[3] = {-std::sin(lon), std::cos(lon), 0.0};
    const double n[3] = {-std::sin(lat) * std::cos(lon), -std::sin(lat) * std::sin(lon),
                         std::cos(lat)};
    double x[3], y[3];
    for (int i = 0; i < 3; i++) {
        x[i] = std::cos(az) * e[i] + std::sin(az) * n[i];
        y[i] = -std::sin(az) * e[i] + std::cos(az) * n[i];
    }
    r[0] = R * std::cos(lat) * std::cos(lon);
    r[1] = R * std::cos(lat) * std::sin(lon);
    r[2] = R * std::sin(lat);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) D[3 * i + j] = 0.5 * (x[i] * x[j] - y[i] * y[j]);
}

// float -> bfloat16, round to nearest even (inputs are finite)
uint16_t bf16_rne(float f)
{
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

float bf16_to_float(uint16_t h)
{
    const uint32_t b = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

bool sample_valid(const ile_ctx *c, const double *s, int64_t N, int64_t i)
{
    double th[7];
    for (int p = 0; p < 7; p++) {
        th[p] = s[p * N + i];
        if (!std::isfinite(th[p])) return false;
    }
    return th[5] > 0.0 && th[4] >= -1.0 && th[4] <= 1.0 &&
           std::fabs(th[6]) <= c->cfg.t_ref_max_s;
}

ile_status check_samples(ile_ctx *c, const double *s, int64_t N)
{
    for (int64_t i = 0; i < N; i++)
        if (!sample_valid(c, s, N, i))
            return fail(c, ILE_E_RANGE,
                        "sample %lld out of range (need finite values, D > 0, "
                        "|cos iota| <= 1, |t_ref| <= %g)",
                        (long long)i, c->cfg.t_ref_max_s);
    return ILE_OK;
}

// Positions per launch of the per-sample terms for N samples.
int64_t terms_cap(int64_t N)
{
    const int64_t n = std::min<int64_t>(std::max<int64_t>(N, 1), ILE_TERMS_CHUNK);
    return (n + 15) & ~(int64_t)15;
}

ile_status ensure_work(ile_ctx *c, int64_t N)
{
    ile_status s;
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    if ((s = ensure(c, c->shifts, n * c->g.n_det * sizeof(int32_t)))) return s;
    if ((s = ensure(c, c->keys, n * sizeof(uint32_t)))) return s;
    if ((s = ensure(c, c->perm, n * sizeof(int32_t)))) return s;
    if ((s = ensure(c, c->hist, (size_t)c->n_buckets * sizeof(uint32_t)))) return s;
    if ((s = ensure(c, c->scan_tmp, (size_t)ile_scan_tmp_words(c->n_buckets) * 4 + 16))) return s;
    if ((s = ensure(c, c->errflag, 16))) return s;
    if ((s = ensure(c, c->red_tmp, 4 * (size_t)ile_reduce_blocks() * sizeof(double)))) return s;
    if ((s = ensure(c, c->res, 8 * sizeof(double)))) return s;
    if (ile_contract_uses_terms(c->cfg.precision, c->tune)) {
        if ((s = ensure(c, c->terms,
                        (size_t)ile_terms_fields(c->g) * terms_cap(N) * sizeof(double))))
            return s;
        if ((s = ensure(c, c->smp_s, n * 7 * sizeof(double)))) return s;
        if ((s = ensure(c, c->sh_s, n * c->g.n_det * sizeof(int32_t)))) return s;
    }
    return ILE_OK;
}

hipEvent_t next_event(ile_ctx *c)
{
    if ((int)c->ev.size() <= c->n_ev_used) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev.push_back(e);
    }
    return c->ev[c->n_ev_used++];
}

// Device scratch of one evaluation: window starts, ordering keys, the sample
// order, the bucket counts and their scan, the reduction's partials.
struct Work {
    int32_t *shifts;
    uint32_t *keys;
    int32_t *perm;
    uint32_t *hist;
    uint32_t *scan_tmp;
    double *red_tmp;
    double *terms;   // per-sample terms of the phased engine, cap positions
    int64_t cap;
    double *smp_s;   // the samples [7][N] and window starts [n_det][N] in tile
    int32_t *sh_s;   // order, for the phased engine's terms pass (or null)
};

Work ctx_work(ile_ctx *c, int64_t N)
{
    return Work{(int32_t *)c->shifts.p, (uint32_t *)c->keys.p, (int32_t *)c->perm.p,
                (uint32_t *)c->hist.p, (uint32_t *)c->scan_tmp.p, (double *)c->red_tmp.p,
                (double *)c->terms.p, terms_cap(N), (double *)c->smp_s.p,
                (int32_t *)c->sh_s.p};
}

// The hot path on device data: window starts and ordering, then the fused
// contraction / time marginalization.  Stream-ordered; allocates nothing.
// timed: bracket the contraction with a pair of the context's events.
ile_status launch_eval(ile_ctx *c, const Work &w, const double *smp, int64_t N, double *out,
                       double *series, bool timed)
{
    if (N <= 0) return ILE_OK;
    const size_t lds_need = ile_contract_lds_bytes(c->g, c->cfg.precision, c->tune);
    if (lds_need > (size_t)c->lds_max)
        return fail(c, ILE_E_UNSUPPORTED,
                    "contraction needs %zu bytes of LDS per workgroup, device has %d",
                    lds_need, c->lds_max);
    hipStream_t st = c->stream;
    HIP_TRY(c, ile_launch_fill_u32(w.hist, 0u, c->n_buckets, st));
    HIP_TRY(c, ile_launch_prep(c->g, smp, N, w.shifts, w.keys, w.hist, c->n_buckets,
                               (int32_t *)c->errflag.p, st));
    // the phased engine's terms pass reads the samples in tile order: the
    // sort moves them there (or, unsorted, they are there already)
    const bool terms = ile_contract_uses_terms(c->cfg.precision, c->tune);
    const double *smp_s = nullptr;
    const int32_t *sh_s = nullptr;
    if (c->sort) {
        HIP_TRY(c, ile_launch_scan(w.hist, c->n_buckets, w.scan_tmp, st));
        if (terms && w.smp_s && w.sh_s) {
            HIP_TRY(c, ile_launch_scatter_copy(w.keys, N, w.hist, w.perm, smp, w.shifts,
                                               c->g.n_det, w.smp_s, w.sh_s, st));
            smp_s = w.smp_s;
            sh_s = w.sh_s;
        } else {
            HIP_TRY(c, ile_launch_scatter(w.keys, N, w.hist, w.perm, st));
        }
    } else {
        HIP_TRY(c, ile_launch_identity(w.perm, N, st));
        smp_s = smp;
        sh_s = w.shifts;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = next_event(c);
        e1 = next_event(c);
        if (!e0 || !e1) return fail(c, ILE_E_DEVICE, "hipEventCreate failed");
        HIP_TRY(c, hipEventRecord(e0, st));
    }
    HIP_TRY(c, ile_launch_contract(c->g, c->cfg.precision, c->tune, smp, N, w.perm, w.shifts,
                                   c->Q.p, (const double *)c->U.p, (const double *)c->V.p,
                                   smp_s, sh_s, (const double *)c->uvt.p, w.terms, w.cap, out,
                                   series, st));
    if (timed) HIP_TRY(c, hipEventRecord(e1, st));
    return ILE_OK;
}

ile_status run_eval(ile_ctx *c, const double *smp, int64_t N, double *out,
                    double *series)
{
    if (N <= 0) return ILE_OK;
    if (N > 0x7fffffff) return fail(c, ILE_E_ARG, "N = %lld exceeds 2^31-1", (long long)N);
    ile_status s = ensure_work(c, N);
    if (s) return s;
    return launch_eval(c, ctx_work(c, N), smp, N, out, series, true);
}

void begin_call(ile_ctx *c)
{
    c->err.clear();
    c->n_ev_used = 0;
}

// Wait for the stream, collect kernel times and the sticky error flag.  The
// flag and the 6 result fields (whatever the call left there) come back to
// pinned host memory with the one wait (fetched_result reads the fields).
ile_status finish_call(ile_ctx *c)
{
    int32_t *hflag = (int32_t *)c->hpin;
    if (c->errflag.p)
        HIP_TRY(c, hipMemcpyAsync(hflag, c->errflag.p, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  c->stream));
    if (c->res.p)
        HIP_TRY(c, hipMemcpyAsync((double *)c->hpin + 1, c->res.p, 6 * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int n = 0;
    for (int i = 0; i + 1 < c->n_ev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) == hipSuccess) {
            tot += ms;
            n++;
        }
    }
    if (n) c->last_ms = tot / n;
    if (c->errflag.p) {
        if (*hflag) {
            HIP_TRY(c, hipMemset(c->errflag.p, 0, sizeof(int32_t)));
            return fail(c, ILE_E_RANGE,
                        "a device-side sample was out of range (its output is NaN)");
        }
    }
    return ILE_OK;
}

// The result fields as of the last finish_call.
void fetched_result(const ile_ctx *c, double r[6])
{
    std::memcpy(r, (const double *)c->hpin + 1, 6 * sizeof(double));
}

ile_status check_ready(ile_ctx *c)
{
    if (!c) return ILE_E_ARG;
    if (!c->have_data) return fail(c, ILE_E_STATE, "ile_set_data has not been called");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    begin_call(c);
    return ILE_OK;
}

}  // namespace

const ile_geom &ile_ctx_geom(const ile_ctx *c) { return c->g; }
const void *ile_ctx_Q(const ile_ctx *c) { return c->Q.p; }
const double *ile_ctx_U(const ile_ctx *c) { return (const double *)c->U.p; }
const double *ile_ctx_V(const ile_ctx *c) { return (const double *)c->V.p; }
ile_precision ile_ctx_precision(const ile_ctx *c) { return c->cfg.precision; }
const double *ile_ctx_uvt(const ile_ctx *c) { return (const double *)c->uvt.p; }
hipStream_t ile_ctx_stream(const ile_ctx *c) { return c->stream; }
int ile_ctx_hist(const ile_ctx *c, const double **P, const double **C)
{
    *P = (const double *)c->hP.p;
    *C = (const double *)c->hC.p;
    return c->hP.p ? c->hist_nb : 0;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char *ile_status_string(ile_status s)
{
    switch (s) {
    case ILE_OK: return "ok";
    case ILE_E_ARG: return "invalid argument";
    case ILE_E_STATE: return "invalid state";
    case ILE_E_RANGE: return "out of range";
    case ILE_E_NUMERIC: return "non-finite or inconsistent data";
    case ILE_E_DEVICE: return "device error";
    case ILE_E_NOMEM: return "out of device memory";
    case ILE_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *ile_last_error(const ile_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

ile_status ile_create(const ile_config *cfg, ile_ctx **out)
{
    if (!out) return ILE_E_ARG;
    *out = nullptr;
    if (!cfg) return ILE_E_ARG;
    if (cfg->n_det < 1 || cfg->n_det > ILE_MAX_DET || cfg->n_lm < 1 ||
        cfg->n_lm > ILE_MAX_LM || !cfg->modes || !(cfg->srate_hz > 0) ||
        cfg->n_t < 1 || cfg->n_t > 65535 || cfg->n_t % 2 == 0 ||
        !(cfg->d_ref_mpc > 0) || !std::isfinite(cfg->gmst_rad) ||
        !(cfg->earth_radius_m > 0) || !(cfg->t_ref_max_s >= 0) ||
        enum_raw(cfg->precision) < ILE_FP64 || enum_raw(cfg->precision) > ILE_BF16)
        return ILE_E_ARG;
    for (int a = 0; a < cfg->n_lm; a++) {
        int l = cfg->modes[a].l, m = cfg->modes[a].m;
        if (l < 2 || l > ILE_LMAX || m < -l || m > l) return ILE_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ILE_E_DEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return ILE_E_ARG;
    ile_ctx *c = new (std::nothrow) ile_ctx();
    if (!c) return ILE_E_NOMEM;
    c->cfg = *cfg;
    c->modes.assign(cfg->modes, cfg->modes + cfg->n_lm);
    c->cfg.modes = c->modes.data();
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete c;
        return ILE_E_DEVICE;
    }
    if (hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              cfg->device) != hipSuccess ||
        scratch_setup(cfg->device) != hipSuccess) {
        delete c;
        return ILE_E_DEVICE;
    }
    // every precision defaults to the matrix cores: the phased engine for
    // FP64 and FP32, the producer/consumer pipeline for BF16 (its only
    // engine), 128 positions per block there (three workgroups per CU)
    c->tune.engine = cfg->precision == ILE_BF16 ? 1 : 3;
    c->tune.threads = cfg->precision == ILE_BF16 ? 128 : 512;
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return ILE_E_DEVICE;
        }
        c->own_stream = true;
    }
    if (hipHostMalloc(&c->hpin, 64, hipHostMallocDefault) != hipSuccess) {
        c->hpin = nullptr;
        ile_destroy(c);
        return ILE_E_DEVICE;
    }
    ile_geom &g = c->g;
    g.n_det = cfg->n_det;
    g.n_lm = cfg->n_lm;
    g.n_t = cfg->n_t;
    g.half = (cfg->n_t - 1) / 2;
    g.dt = 1.0 / cfg->srate_hz;
    g.d_ref = cfg->d_ref_mpc;
    g.gmst = cfg->gmst_rad;
    g.t_ref_max = cfg->t_ref_max_s;
    if (!build_ylm_table(g, c->modes)) {
        ile_destroy(c);
        return ILE_E_UNSUPPORTED;
    }
    *out = c;
    return ILE_OK;
}

ile_status ile_set_data(ile_ctx *c, const double *Q, int64_t n_q, double t0_s,
                        const double *U, const double *V, const ile_detector *dets)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (!Q || !U || !V || !dets) return fail(c, ILE_E_ARG, "null pointer");
    const int nd = c->cfg.n_det, nl = c->cfg.n_lm;
    if (n_q < c->cfg.n_t || n_q > (int64_t)0x7fffffff / 2)
        return fail(c, ILE_E_ARG, "n_q = %lld invalid", (long long)n_q);
    if (!std::isfinite(t0_s)) return fail(c, ILE_E_ARG, "t0 not finite");
    const size_t nQ = (size_t)nd * nl * n_q, nUV = (size_t)nd * nl * nl;
    for (size_t i = 0; i < 2 * nQ; i++)
        if (!std::isfinite(Q[i])) return fail(c, ILE_E_NUMERIC, "Q[%zu] not finite", i / 2);
    for (size_t i = 0; i < 2 * nUV; i++)
        if (!std::isfinite(U[i]) || !std::isfinite(V[i]))
            return fail(c, ILE_E_NUMERIC, "U or V entry %zu not finite", i / 2);
    for (int k = 0; k < nd; k++) {
        double mx = 0.0;
        for (int i = 0; i < nl * nl; i++) {
            const double *u = U + 2 * ((size_t)k * nl * nl + i);
            mx = std::max(mx, std::hypot(u[0], u[1]));
        }
        for (int a = 0; a < nl; a++)
            for (int b = 0; b < nl; b++) {
                const double *uab = U + 2 * (((size_t)k * nl + a) * nl + b);
                const double *uba = U + 2 * (((size_t)k * nl + b) * nl + a);
                if (std::fabs(uab[0] - uba[0]) > 1e-12 * mx ||
                    std::fabs(uab[1] + uba[1]) > 1e-12 * mx)
                    return fail(c, ILE_E_NUMERIC, "U[%d] not Hermitian at (%d,%d)", k, a, b);
            }
    }
    ile_geom &g = c->g;
    for (int k = 0; k < nd; k++) {
        const ile_detector &d = dets[k];
        if (!std::isfinite(d.lat_deg) || !std::isfinite(d.lon_deg) ||
            !std::isfinite(d.xarm_az_deg) || std::fabs(d.lat_deg) > 90.0)
            return fail(c, ILE_E_ARG, "detector %d invalid", k);
        detector_frame(d, c->cfg.earth_radius_m, g.r[k], g.D[k]);
    }
    g.n_q = (int)n_q;
    g.s_max = (int)(n_q - c->cfg.n_t);
    g.t0 = t0_s;
    // every window reachable with |t_ref| <= t_ref_max must lie in Q
    const double reach = c->cfg.t_ref_max_s + c->cfg.earth_radius_m / kC;
    const double xlo = (-reach - t0_s) / g.dt, xhi = (reach - t0_s) / g.dt;
    const int64_t slo = (int64_t)std::floor(xlo + 0.5) - g.half - 1;
    const int64_t shi = (int64_t)std::floor(xhi + 0.5) - g.half + 1;
    if (slo < 0 || shi > g.s_max)
        return fail(c, ILE_E_RANGE,
                    "Q too short: windows reach indices [%lld, %lld] but Q has %lld",
                    (long long)slo, (long long)(shi + c->cfg.n_t - 1), (long long)n_q);
    // ordering key: cells of 2^shift samples over [slo, shi], <= 21 bits
    const int64_t width = shi - slo + 1;
    g.key_dims = std::min(nd, 3);
    int shift = 4, bits = 0;
    for (;;) {
        int64_t cells = (width + (1 << shift) - 1) >> shift;
        bits = 0;
        while ((1ll << bits) < cells) bits++;
        if (bits * g.key_dims <= 21) break;
        shift++;
    }
    g.key_shift = shift;
    g.key_bits = bits;
    for (int d = 0; d < 3; d++) g.key_lo[d] = (int)slo;
    c->n_buckets = (1u << (bits * g.key_dims)) + 1u;

    ile_status s;
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    // device layout: planar rows per detector, row 2a = Re Q_a, 2a+1 = Im Q_a,
    // padded with zero rows to 4 * ksp_of(n_lm) (the matrix-core K steps)
    const size_t rp = (size_t)4 * ksp_of(nl);
    const size_t nQd = (size_t)nd * rp * n_q;
    const size_t qe = c->cfg.precision == ILE_FP64 ? 8 : 4;
    const size_t kb = (size_t)32 * ksb_of(nl);   // BF16 rows per position
    const size_t q_bytes = c->cfg.precision == ILE_BF16 ? (size_t)nd * n_q * kb * 2 : nQd * qe;
    if ((s = ensure(c, c->Q, q_bytes))) return s;
    if ((s = ensure(c, c->U, nUV * 16))) return s;
    if ((s = ensure(c, c->V, nUV * 16))) return s;
    if (c->cfg.precision == ILE_FP64) {
        std::vector<double> h(nQd, 0.0);
        for (int k = 0; k < nd; k++)
            for (int a = 0; a < nl; a++)
                for (int64_t i = 0; i < n_q; i++) {
                    const double *q = Q + 2 * (((size_t)k * nl + a) * n_q + i);
                    h[((size_t)k * rp + 2 * a) * n_q + i] = q[0];
                    h[((size_t)k * rp + 2 * a + 1) * n_q + i] = q[1];
                }
        HIP_TRY(c, hipMemcpy(c->Q.p, h.data(), nQd * 8, hipMemcpyHostToDevice));
    } else if (c->cfg.precision == ILE_BF16) {
        // K-contiguous per position: [Q_hi rows; Q_lo rows; Q_hi rows; zeros]
        std::vector<uint16_t> h((size_t)nd * n_q * kb, 0);
        const size_t R = 2 * (size_t)nl;
        for (int k = 0; k < nd; k++)
            for (int a = 0; a < nl; a++)
                for (int64_t i = 0; i < n_q; i++) {
                    const double *q = Q + 2 * (((size_t)k * nl + a) * n_q + i);
                    uint16_t *row = &h[((size_t)k * n_q + i) * kb];
                    for (int c2 = 0; c2 < 2; c2++) {
                        const uint16_t hi = bf16_rne((float)q[c2]);
                        const uint16_t lo = bf16_rne((float)(q[c2] - (double)bf16_to_float(hi)));
                        const size_t r = 2 * a + c2;
                        row[r] = hi;
                        row[R + r] = lo;
                        row[2 * R + r] = hi;
                    }
                }
        HIP_TRY(c, hipMemcpy(c->Q.p, h.data(), h.size() * 2, hipMemcpyHostToDevice));
    } else {
        std::vector<float> h(nQd, 0.0f);
        for (int k = 0; k < nd; k++)
            for (int a = 0; a < nl; a++)
                for (int64_t i = 0; i < n_q; i++) {
                    const double *q = Q + 2 * (((size_t)k * nl + a) * n_q + i);
                    h[((size_t)k * rp + 2 * a) * n_q + i] = (float)q[0];
                    h[((size_t)k * rp + 2 * a + 1) * n_q + i] = (float)q[1];
                }
        HIP_TRY(c, hipMemcpy(c->Q.p, h.data(), nQd * 4, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->U.p, U, nUV * 16, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->V.p, V, nUV * 16, hipMemcpyHostToDevice));
    // the Hermitian part of U and the symmetric part of V: the only parts
    // the quadratic term of Eq. (7) sees (Re(Y^H U Y) = Y^H U_h Y,
    // Y^T V Y = Y^T V_s Y)
    // (upper triangles, row by row, U_h and V_s interleaved per entry)
    {
        std::vector<double> t;
        t.reserve((size_t)nd * nl * (nl + 1) * 2);
        for (int k = 0; k < nd; k++)
            for (int a = 0; a < nl; a++)
                for (int b = a; b < nl; b++) {
                    const size_t e = ((size_t)k * nl + a) * nl + b, f = ((size_t)k * nl + b) * nl + a;
                    t.push_back(0.5 * (U[2 * e] + U[2 * f]));
                    t.push_back(0.5 * (U[2 * e + 1] - U[2 * f + 1]));
                    t.push_back(0.5 * (V[2 * e] + V[2 * f]));
                    t.push_back(0.5 * (V[2 * e + 1] + V[2 * f + 1]));
                }
        if ((s = ensure(c, c->uvt, t.size() * sizeof(double)))) return s;
        HIP_TRY(c, hipMemcpy(c->uvt.p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if ((s = ensure(c, c->errflag, 16))) return s;
    HIP_TRY(c, hipMemset(c->errflag.p, 0, 16));
    c->have_data = true;
    return ILE_OK;
}

ile_status ile_inject(ile_ctx *c, const double *h_lm, int64_t n_q, double t0_s,
                      const ile_detector *dets, const double *theta, double snr,
                      double *rho2_out, double *d_inj_out, double *Q_out, double *U_out,
                      double *V_out)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (!h_lm || !dets || !theta) return fail(c, ILE_E_ARG, "null pointer");
    const int nd = c->cfg.n_det, nl = c->cfg.n_lm;
    if (n_q < c->cfg.n_t || n_q > (1 << 24)) return fail(c, ILE_E_ARG, "n_q out of range");
    for (int p = 0; p < 7; p++)
        if (!std::isfinite(theta[p])) return fail(c, ILE_E_ARG, "theta not finite");
    if (!(theta[5] > 0) || std::fabs(theta[4]) > 1.0 || !(snr >= 0) || !std::isfinite(snr))
        return fail(c, ILE_E_ARG, "bad injected parameters or snr");
    for (size_t i = 0; i < (size_t)2 * nl * n_q; i++)
        if (!std::isfinite(h_lm[i])) return fail(c, ILE_E_NUMERIC, "h_lm not finite");
    ile_geom g = c->g;
    for (int k = 0; k < nd; k++) {
        const ile_detector &d = dets[k];
        if (!std::isfinite(d.lat_deg) || !std::isfinite(d.lon_deg) ||
            !std::isfinite(d.xarm_az_deg) || std::fabs(d.lat_deg) > 90.0)
            return fail(c, ILE_E_ARG, "detector %d invalid", k);
        detector_frame(d, c->cfg.earth_radius_m, g.r[k], g.D[k]);
    }
    g.n_q = (int)n_q;
    g.t0 = t0_s;
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    const size_t n = (size_t)n_q;
    DevBuf hd, th, dd, Qd, Ud, Vd;
    auto cleanup = [&]() {
        for (DevBuf *b : {&hd, &th, &dd, &Qd, &Ud, &Vd}) release(*b);
    };
    ile_status s = ILE_OK;
    if ((s = ensure(c, hd, 16 * nl * n)) || (s = ensure(c, th, 7 * 8)) ||
        (s = ensure(c, dd, 8 * nd * n)) || (s = ensure(c, Qd, 16 * (size_t)nd * nl * n)) ||
        (s = ensure(c, Ud, 16 * (size_t)nl * nl)) || (s = ensure(c, Vd, 16 * (size_t)nl * nl))) {
        cleanup();
        return s;
    }
    std::vector<double> d((size_t)nd * n), Q((size_t)2 * nd * nl * n),
        U1((size_t)2 * nl * nl), V1((size_t)2 * nl * nl);
    hipError_t e = hipMemcpyAsync(hd.p, h_lm, 16 * nl * n, hipMemcpyHostToDevice, c->stream);
    if (!e) e = hipMemcpyAsync(th.p, theta, 7 * 8, hipMemcpyHostToDevice, c->stream);
    if (!e) e = ile_launch_inject(g, (const double *)hd.p, (int)n, (const double *)th.p,
                                  (double *)dd.p, c->stream);
    if (!e) e = hipStreamSynchronize(c->stream);
    if (!e) e = hipMemcpy(d.data(), dd.p, 8 * d.size(), hipMemcpyDeviceToHost);
    long double r2 = 0.0L;
    for (double v : d) r2 += (long double)v * v;
    const double rho2 = (double)r2;
    const double scale = (snr > 0 && rho2 > 0) ? snr / std::sqrt(rho2) : 1.0;
    if (!e) e = ile_launch_inject_qv(nd, nl, (int)n, (const double *)hd.p, (const double *)dd.p,
                                     scale, (double *)Qd.p, (double *)Ud.p, (double *)Vd.p,
                                     c->stream);
    if (!e) e = hipStreamSynchronize(c->stream);
    if (!e) e = hipMemcpy(Q.data(), Qd.p, 8 * Q.size(), hipMemcpyDeviceToHost);
    if (!e) e = hipMemcpy(U1.data(), Ud.p, 8 * U1.size(), hipMemcpyDeviceToHost);
    if (!e) e = hipMemcpy(V1.data(), Vd.p, 8 * V1.size(), hipMemcpyDeviceToHost);
    cleanup();
    if (e) return fail(c, ILE_E_DEVICE, "injection: %s", hipGetErrorString(e));
    // white noise: the same U, V at every detector; U exactly Hermitian
    std::vector<double> U((size_t)2 * nd * nl * nl), V(U.size());
    for (int k = 0; k < nd; k++)
        for (int a = 0; a < nl; a++)
            for (int b = 0; b < nl; b++) {
                const size_t o = 2 * (((size_t)k * nl + a) * nl + b), ab = 2 * ((size_t)a * nl + b),
                             ba = 2 * ((size_t)b * nl + a);
                U[o] = 0.5 * (U1[ab] + U1[ba]);
                U[o + 1] = 0.5 * (U1[ab + 1] - U1[ba + 1]);
                V[o] = V1[ab];
                V[o + 1] = V1[ab + 1];
            }
    if ((s = ile_set_data(c, Q.data(), n_q, t0_s, U.data(), V.data(), dets))) return s;
    if (rho2_out) *rho2_out = rho2 * scale * scale;
    if (d_inj_out) *d_inj_out = theta[5] / scale;
    if (Q_out) memcpy(Q_out, Q.data(), 8 * Q.size());
    if (U_out) memcpy(U_out, U.data(), 8 * U.size());
    if (V_out) memcpy(V_out, V.data(), 8 * V.size());
    return ILE_OK;
}

// Q, U, V of Eq. (8) from frequency-domain series (Eq. (2) on the FFT grid):
// the band-weighted products, an inverse FFT per (detector, mode) row and the
// U, V sums, all on the device.  Blocking.
ile_status ile_qvu_fd_dev(ile_ctx *c, const double *h_f, const double *d_f, const double *psd,
                          int64_t n_q, double df, double f_min, double f_max, double t0_s,
                          double *Q, double *U, double *V)
{
    if (!c) return ILE_E_ARG;
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    begin_call(c);
    if (!h_f || !d_f || !psd || !Q || !U || !V) return fail(c, ILE_E_ARG, "null pointer");
    if (n_q < 2 || n_q > ((int64_t)1 << 20) || (n_q & (n_q - 1)))
        return fail(c, ILE_E_UNSUPPORTED, "n_q = %lld is not a power of two in [2, 2^20]",
                    (long long)n_q);
    if (!(df > 0) || !std::isfinite(df) || !std::isfinite(t0_s) || std::isnan(f_min) ||
        std::isnan(f_max) || !(f_max > f_min))
        return fail(c, ILE_E_ARG, "bad df, band or t0");
    const int nd = c->cfg.n_det, nl = c->cfg.n_lm, rows = nd * nl;
    ile_status s;
    if ((s = ensure(c, c->fd_tmp, (size_t)rows * n_q * 16))) return s;
    if ((s = ensure(c, c->fd_flag, 16))) return s;
    hipStream_t st = c->stream;
    int32_t *flag = (int32_t *)c->fd_flag.p;
    // the inverse FFT ends in Q: start in the scratch buffer when the number
    // of its kernels (one for n_q <= 1024, else two) is odd
    const bool odd = ile_fft_passes(n_q) & 1;
    double *a = odd ? (double *)c->fd_tmp.p : Q, *b = odd ? Q : (double *)c->fd_tmp.p, *res = nullptr;
    HIP_TRY(c, hipMemsetAsync(flag, 0, sizeof(int32_t), st));
    HIP_TRY(c, ile_launch_fd_prod(h_f, d_f, psd, n_q, nd, nl, df, f_min, f_max, t0_s, a, flag, st));
    hipEvent_t e0 = next_event(c), e1 = next_event(c);
    if (!e0 || !e1) return fail(c, ILE_E_DEVICE, "hipEventCreate failed");
    HIP_TRY(c, hipEventRecord(e0, st));
    HIP_TRY(c, ile_launch_ifft_rows(a, b, n_q, rows, &res, st));
    HIP_TRY(c, hipEventRecord(e1, st));
    if (res != Q) return fail(c, ILE_E_DEVICE, "internal: FFT result buffer");
    HIP_TRY(c, ile_launch_uv_fd(h_f, psd, n_q, nd, nl, df, f_min, f_max, U, V, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) c->last_ms = ms;
    c->n_ev_used = 0;
    int32_t f = 0;
    HIP_TRY(c, hipMemcpy(&f, flag, sizeof(f), hipMemcpyDeviceToHost));
    if (f) return fail(c, ILE_E_NUMERIC, "non-finite input or non-positive spectrum in the band");
    return ILE_OK;
}

ile_status ile_set_data_fd(ile_ctx *c, const double *h_f, const double *d_f, const double *psd,
                           int64_t n_q, double df, double f_min, double f_max, double t0_s,
                           const ile_detector *dets, double *Q_out, double *U_out,
                           double *V_out)
{
    if (!c) return ILE_E_ARG;
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    begin_call(c);
    if (!h_f || !d_f || !psd || !dets) return fail(c, ILE_E_ARG, "null pointer");
    if (n_q < 2 || n_q > ((int64_t)1 << 20) || (n_q & (n_q - 1)))
        return fail(c, ILE_E_UNSUPPORTED, "n_q = %lld is not a power of two in [2, 2^20]",
                    (long long)n_q);
    const int nd = c->cfg.n_det, nl = c->cfg.n_lm;
    const size_t nh = (size_t)2 * nl * n_q, ndd = (size_t)2 * nd * n_q, np_ = (size_t)nd * n_q;
    const size_t nQ = (size_t)2 * nd * nl * n_q, nUV = (size_t)2 * nd * nl * nl;
    ile_status s;
    if ((s = ensure(c, c->fd_in, (nh + ndd + np_) * sizeof(double)))) return s;
    if ((s = ensure(c, c->fd_out, (nQ + 2 * nUV) * sizeof(double)))) return s;
    double *dh = (double *)c->fd_in.p, *dd = dh + nh, *dp = dd + ndd;
    double *dQ = (double *)c->fd_out.p, *dU = dQ + nQ, *dV = dU + nUV;
    HIP_TRY(c, hipMemcpy(dh, h_f, nh * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dd, d_f, ndd * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dp, psd, np_ * sizeof(double), hipMemcpyHostToDevice));
    if ((s = ile_qvu_fd_dev(c, dh, dd, dp, n_q, df, f_min, f_max, t0_s, dQ, dU, dV))) return s;
    std::vector<double> Q(nQ), U(nUV), V(nUV);
    HIP_TRY(c, hipMemcpy(Q.data(), dQ, nQ * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(U.data(), dU, nUV * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(V.data(), dV, nUV * sizeof(double), hipMemcpyDeviceToHost));
    if ((s = ile_set_data(c, Q.data(), n_q, t0_s, U.data(), V.data(), dets))) return s;
    if (Q_out) memcpy(Q_out, Q.data(), nQ * sizeof(double));
    if (U_out) memcpy(U_out, U.data(), nUV * sizeof(double));
    if (V_out) memcpy(V_out, V.data(), nUV * sizeof(double));
    return ILE_OK;
}

// Surrogate (linear-basis) form, Sec. V: the context's n_lm "modes" are
// basis functions e_b with Q, U, V their overlaps; each joint sample carries
// lambda in row 7, and z = C(lambda) Y takes the place of the harmonics.
ile_status ile_rom_set(ile_ctx *c, const ile_mode *modes, int32_t n_lm, int32_t n_pow,
                       const double *A)
{
    if (!c) return ILE_E_ARG;
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    begin_call(c);
    if (!modes || !A) return fail(c, ILE_E_ARG, "null pointer");
    if (n_lm < 1 || n_lm > ILE_MAX_LM || n_pow < 1 || n_pow > 8)
        return fail(c, ILE_E_ARG, "n_lm = %d or n_pow = %d out of range", n_lm, n_pow);
    for (int a = 0; a < n_lm; a++)
        if (modes[a].l < 2 || modes[a].l > 6 || std::abs(modes[a].m) > modes[a].l)
            return fail(c, ILE_E_ARG, "mode %d invalid", a);
    ile_geom gp{};
    gp.n_lm = n_lm;
    if (!build_ylm_table(gp, std::vector<ile_mode>(modes, modes + n_lm)))
        return fail(c, ILE_E_ARG, "mode list too long");
    const size_t na = (size_t)2 * n_lm * c->cfg.n_lm * n_pow;
    for (size_t i = 0; i < na; i++)
        if (!std::isfinite(A[i])) return fail(c, ILE_E_NUMERIC, "A[%zu] not finite", i / 2);
    ile_status s;
    if ((s = ensure(c, c->rom_A, na * sizeof(double)))) return s;
    HIP_TRY(c, hipMemcpy(c->rom_A.p, A, na * sizeof(double), hipMemcpyHostToDevice));
    c->rom_g = gp;
    c->rom_pow = n_pow;
    return ILE_OK;
}

static ile_status rom_eval_impl(ile_ctx *c, const double *smp, int64_t N, double *out)
{
    ile_status s;
    const int nb = c->cfg.n_lm;
    if ((s = ensure(c, c->rom_Z, (size_t)std::max<int64_t>(N, 1) * nb * 2 * sizeof(double))))
        return s;
    if ((s = ensure_work(c, N))) return s;
    HIP_TRY(c, ile_launch_rom_z(c->rom_g, smp, N, (const double *)c->rom_A.p, nb, c->rom_pow,
                                (double *)c->rom_Z.p, (int32_t *)c->errflag.p, c->stream));
    c->g.ext_y = (const double2 *)c->rom_Z.p;
    s = run_eval(c, smp, N, out, nullptr);
    c->g.ext_y = nullptr;
    return s;
}

ile_status ile_rom_eval_dev(ile_ctx *c, const double *smp, int64_t N, double *out)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (!c->rom_pow) return fail(c, ILE_E_STATE, "ile_rom_set has not been called");
    if (N < 0 || (N > 0 && (!smp || !out))) return fail(c, ILE_E_ARG, "bad N or pointer");
    if (N == 0) return ILE_OK;
    return rom_eval_impl(c, smp, N, out);
}

ile_status ile_rom_integrate_dev(ile_ctx *c, const double *smp, const double *lp,
                                 const double *lq, int64_t N, double *res)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (!c->rom_pow) return fail(c, ILE_E_STATE, "ile_rom_set has not been called");
    if (N < 0 || !res || (N > 0 && !smp)) return fail(c, ILE_E_ARG, "bad N or pointer");
    if ((s = ensure(c, c->out, (size_t)std::max<int64_t>(N, 1) * sizeof(double)))) return s;
    if ((s = ensure(c, c->parts, 8 * sizeof(double)))) return s;
    if ((s = ensure_work(c, N))) return s;
    if (N > 0 && (s = rom_eval_impl(c, smp, N, (double *)c->out.p))) return s;
    HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, lp, lq, N, (double *)c->red_tmp.p,
                                 (double *)c->parts.p, c->stream));
    HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, 1, res, c->stream));
    return ILE_OK;
}

ile_status ile_eval_dev(ile_ctx *c, const double *smp, int64_t N, double *out)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N < 0 || (N > 0 && (!smp || !out))) return fail(c, ILE_E_ARG, "bad N or pointer");
    return run_eval(c, smp, N, out, nullptr);
}

static ile_status eval_host(ile_ctx *c, const double *samples, int64_t N,
                            double *out, bool series)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N < 0 || (N > 0 && (!samples || !out))) return fail(c, ILE_E_ARG, "bad N or pointer");
    if (N == 0) return ILE_OK;
    if ((s = check_samples(c, samples, N))) return s;
    if ((s = ensure(c, c->smp, (size_t)N * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->out, (size_t)N * sizeof(double)))) return s;
    size_t ser_bytes = series ? (size_t)N * c->cfg.n_t * sizeof(double) : 0;
    if (series && (s = ensure(c, c->series, ser_bytes))) return s;
    HIP_TRY(c, hipMemcpyAsync(c->smp.p, samples, (size_t)N * 7 * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));
    if ((s = run_eval(c, (const double *)c->smp.p, N, (double *)c->out.p,
                      series ? (double *)c->series.p : nullptr)))
        return s;
    if ((s = finish_call(c))) return s;
    if (series)
        HIP_TRY(c, hipMemcpy(out, c->series.p, ser_bytes, hipMemcpyDeviceToHost));
    else
        HIP_TRY(c, hipMemcpy(out, c->out.p, (size_t)N * sizeof(double),
                             hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_eval(ile_ctx *c, const double *samples, int64_t N, double *out)
{
    return eval_host(c, samples, N, out, false);
}

ile_status ile_eval_series(ile_ctx *c, const double *samples, int64_t N, double *out)
{
    return eval_host(c, samples, N, out, true);
}

static ile_status integrate_dev_impl(ile_ctx *c, const double *smp, const double *lp,
                                     const double *lq, int64_t N, double *res)
{
    ile_status s;
    if ((s = ensure(c, c->out, (size_t)std::max<int64_t>(N, 1) * sizeof(double)))) return s;
    if ((s = ensure(c, c->parts, 8 * sizeof(double)))) return s;
    if ((s = run_eval(c, smp, N, (double *)c->out.p, nullptr))) return s;
    HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, lp, lq, N,
                                 (double *)c->red_tmp.p, (double *)c->parts.p, c->stream));
    HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, 1, res, c->stream));
    return ILE_OK;
}

ile_status ile_integrate_dev(ile_ctx *c, const double *smp, const double *lp,
                             const double *lq, int64_t N, double *res)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N < 0 || !res || (N > 0 && !smp)) return fail(c, ILE_E_ARG, "bad N or pointer");
    if ((s = ensure_work(c, N))) return s;
    return integrate_dev_impl(c, smp, lp, lq, N, res);
}

ile_status ile_integrate_dev_noalloc(ile_ctx *c, const double *smp, const double *lp,
                                     const double *lq, int64_t N, double *res)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N < 0 || !res || (N > 0 && !smp)) return fail(c, ILE_E_ARG, "bad N or pointer");
    if (N > ILE_NOALLOC_MAX_N)
        return fail(c, ILE_E_ARG, "N = %lld exceeds the allocation-free limit of %lld samples",
                    (long long)N, (long long)ILE_NOALLOC_MAX_N);
    unsigned char *base = scratch_of(c->cfg.device);
    if (!base || !c->errflag.p)
        return fail(c, ILE_E_STATE, "no workspace on device %d", c->cfg.device);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        return p;
    };
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    double *out = (double *)take(n * sizeof(double));
    Work w;
    w.shifts = (int32_t *)take(n * c->g.n_det * sizeof(int32_t));
    w.keys = (uint32_t *)take(n * sizeof(uint32_t));
    w.perm = (int32_t *)take(n * sizeof(int32_t));
    w.hist = (uint32_t *)take((size_t)c->n_buckets * sizeof(uint32_t));
    w.scan_tmp = (uint32_t *)take((size_t)ile_scan_tmp_words(c->n_buckets) * 4 + 16);
    w.red_tmp = (double *)take(4 * (size_t)ile_reduce_blocks() * sizeof(double));
    w.cap = terms_cap(N);
    w.terms = (double *)take((size_t)ile_terms_fields(c->g) * w.cap * sizeof(double));
    w.smp_s = (double *)take(n * 7 * sizeof(double));
    w.sh_s = (int32_t *)take(n * c->g.n_det * sizeof(int32_t));
    double *parts = (double *)take(8 * sizeof(double));
    if (off > kNoAllocBytes)
        return fail(c, ILE_E_UNSUPPORTED, "workspace needs %zu bytes, the fixed array has %zu",
                    off, kNoAllocBytes);
    if ((s = launch_eval(c, w, smp, N, out, nullptr, false))) return s;
    HIP_TRY(c, ile_launch_reduce(out, lp, lq, N, w.red_tmp, parts, c->stream));
    HIP_TRY(c, ile_launch_finish(parts, 1, res, c->stream));
    return ILE_OK;
}

static void copy_result(const double *r, ile_result *out)
{
    out->ln_L_marg = r[0];
    out->n_eff = r[1];
    out->n_eff_kish = r[2];
    out->sigma_ln_L = r[3];
    out->max_ln_L = r[4];
    out->n_samples = (int64_t)r[5];
}

ile_status ile_integrate(ile_ctx *c, const double *samples, const double *ln_p,
                         const double *ln_q, int64_t N, ile_result *out)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N < 0 || !out || (N > 0 && (!samples || !ln_p || !ln_q)))
        return fail(c, ILE_E_ARG, "bad N or pointer");
    if ((s = check_samples(c, samples, N))) return s;
    for (int64_t i = 0; i < N; i++)
        if (std::isnan(ln_p[i]) || std::isnan(ln_q[i]) || ln_q[i] == -INFINITY ||
            ln_p[i] == INFINITY)
            return fail(c, ILE_E_RANGE, "ln_p/ln_q of sample %lld invalid", (long long)i);
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    if ((s = ensure(c, c->smp, n * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnp, n * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnq, n * sizeof(double)))) return s;
    if ((s = ensure_work(c, N))) return s;
    if (N > 0) {
        HIP_TRY(c, hipMemcpyAsync(c->smp.p, samples, (size_t)N * 7 * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->lnp.p, ln_p, (size_t)N * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->lnq.p, ln_q, (size_t)N * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    }
    if ((s = integrate_dev_impl(c, (const double *)c->smp.p, (const double *)c->lnp.p,
                                (const double *)c->lnq.p, N, (double *)c->res.p)))
        return s;
    if ((s = finish_call(c))) return s;
    double r[6];
    fetched_result(c, r);
    copy_result(r, out);
    return ILE_OK;
}

ile_status ile_draw_prior_dev(ile_ctx *c, uint64_t seed, int64_t first, int64_t N,
                              double d_min, double d_max, double *smp, int64_t ld,
                              double *ln_p)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (N < 0 || first < 0 || (N > 0 && !smp) || ld < N || !(d_min > 0) ||
        !(d_max > d_min) || !std::isfinite(d_max))
        return fail(c, ILE_E_ARG, "bad prior-draw arguments");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    HIP_TRY(c, ile_launch_prior(seed, first, N, d_min, d_max, c->cfg.t_ref_max_s, smp,
                                ld, ln_p, c->stream));
    return ILE_OK;
}

// Extrinsic posterior harvest (Sec. V; Eq. (3) at fixed intrinsic
// parameters): sample weights and their prefix sums, one inverse-CDF pick per
// draw, then the per-bin series of the picked samples in chunks of at most
// 2 GiB and one bin pick per draw.
ile_status ile_harvest_dev(ile_ctx *c, const double *smp, const double *lp, const double *lq,
                           int64_t N, const double *u, int64_t n_out, int64_t *idx,
                           int32_t *bins, double *theta, double *result)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N <= 0 || n_out < 0 || !smp || (n_out > 0 && (!u || !idx || !bins)))
        return fail(c, ILE_E_ARG, "bad N, n_out or pointer");
    if (N > 0x7fffffff) return fail(c, ILE_E_ARG, "N = %lld exceeds 2^31-1", (long long)N);
    if (n_out == 0) return ILE_OK;
    const int n_t = c->cfg.n_t, nb = ile_hv_parts();
    const int64_t m_max = c->hv_rows > 0 ? c->hv_rows
                                          : std::max<int64_t>(1, ((int64_t)1 << 31) / ((int64_t)n_t * 8));
    const int64_t m_cap = std::min<int64_t>(m_max, n_out);
    hipStream_t st = c->stream;
    if ((s = ensure(c, c->out, (size_t)std::max<int64_t>(N, m_cap) * sizeof(double)))) return s;
    if ((s = ensure(c, c->hv_w, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c, c->hv_cdf, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c, c->hv_ws, ile_mdn_fit_ws_doubles() * sizeof(double)))) return s;
    if ((s = ensure(c, c->hv_part, (size_t)(nb + 1) * sizeof(double)))) return s;
    if ((s = ensure(c, c->hv_flag, 16))) return s;
    if ((s = ensure(c, c->hv_sel, (size_t)m_cap * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->series, (size_t)m_cap * n_t * sizeof(double)))) return s;
    int32_t *flag = (int32_t *)c->hv_flag.p;
    double *lnL = (double *)c->out.p, *w = (double *)c->hv_w.p, *cdf = (double *)c->hv_cdf.p;
    HIP_TRY(c, hipMemsetAsync(flag, 0, sizeof(int32_t), st));
    if ((s = run_eval(c, smp, N, lnL, nullptr))) return s;
    if (result) {
        if ((s = ensure(c, c->parts, 8 * sizeof(double)))) return s;
        HIP_TRY(c, ile_launch_reduce(lnL, lp, lq, N, (double *)c->red_tmp.p,
                                     (double *)c->parts.p, st));
        HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, 1, result, st));
    }
    HIP_TRY(c, ile_launch_hv_weights(lnL, lp, lq, N, w, (double *)c->hv_part.p, flag, st));
    HIP_TRY(c, ile_launch_mdn_cdf(w, N, cdf, (double *)c->hv_ws.p, st));
    HIP_TRY(c, ile_launch_hv_pick(cdf, N, u, n_out, idx, flag, st));
    if ((s = finish_call(c))) return s;
    int32_t f = 0;
    HIP_TRY(c, hipMemcpy(&f, flag, sizeof(f), hipMemcpyDeviceToHost));
    if (f & 1) return fail(c, ILE_E_RANGE, "ln_p/ln_q invalid (NaN, ln p = +inf or ln q = -inf)");
    if (f & 4) return fail(c, ILE_E_RANGE, "a uniform of u lies outside [0, 1)");
    if (f & 2) return fail(c, ILE_E_NUMERIC, "no sample has a finite positive weight");
    double *sel = (double *)c->hv_sel.p, *ser = (double *)c->series.p;
    for (int64_t k0 = 0; k0 < n_out; k0 += m_cap) {
        const int64_t m = std::min<int64_t>(m_cap, n_out - k0);
        HIP_TRY(c, ile_launch_hv_gather(smp, N, idx + k0, m, sel, st));
        if ((s = run_eval(c, sel, m, lnL, ser))) return s;
        HIP_TRY(c, ile_launch_hv_bin(ser, m, n_t, u + n_out + k0, sel, c->cfg.srate_hz,
                                     bins + k0, theta ? theta + k0 : nullptr, n_out, st));
    }
    return finish_call(c);
}

ile_status ile_run_prior(ile_ctx *c, uint64_t seed, int64_t N, int64_t chunk,
                         double d_min, double d_max, ile_result *out)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (N <= 0 || !out || !(d_min > 0) || !(d_max > d_min) || !std::isfinite(d_max))
        return fail(c, ILE_E_ARG, "bad run arguments");
    if (chunk <= 0 || chunk > N) chunk = N;
    const int64_t n_chunks = (N + chunk - 1) / chunk;
    if (n_chunks > 1 << 20) return fail(c, ILE_E_ARG, "too many chunks");
    if ((s = ensure(c, c->smp, (size_t)chunk * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->out, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->parts, (size_t)n_chunks * 5 * sizeof(double)))) return s;
    if ((s = ensure_work(c, chunk))) return s;
    // the proposal is the prior: ln p - ln q = 0, so no density is needed
    for (int64_t ci = 0; ci < n_chunks; ci++) {
        const int64_t first = ci * chunk, n = std::min(chunk, N - first);
        HIP_TRY(c, ile_launch_prior(seed, first, n, d_min, d_max, c->cfg.t_ref_max_s,
                                    (double *)c->smp.p, n, nullptr, c->stream));
        if ((s = run_eval(c, (const double *)c->smp.p, n, (double *)c->out.p, nullptr)))
            return s;
        HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, nullptr, nullptr, n,
                                     (double *)c->red_tmp.p,
                                     (double *)c->parts.p + 5 * ci, c->stream));
    }
    HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, (int)n_chunks,
                                 (double *)c->res.p, c->stream));
    if ((s = finish_call(c))) return s;
    double r[6];
    fetched_result(c, r);
    copy_result(r, out);
    return ILE_OK;
}

static ile_status hist_init(ile_ctx *c, int nb, bool reset)
{
    if (nb < 2 || nb > ILE_MAX_BINS || nb > ile_hist_max_bins())
        return fail(c, ILE_E_ARG, "n_bins = %d outside [2, %d]", nb, ILE_MAX_BINS);
    ile_status s;
    if ((s = ensure(c, c->hP, 2 * (size_t)ILE_MAX_BINS * sizeof(double)))) return s;
    if ((s = ensure(c, c->hC, 2 * (size_t)(ILE_MAX_BINS + 1) * sizeof(double)))) return s;
    if (reset || c->hist_nb != nb) {
        HIP_TRY(c, ile_launch_hist_uniform(nb, (double *)c->hP.p, (double *)c->hC.p, c->stream));
        c->hist_nb = nb;
    }
    return ILE_OK;
}

ile_status ile_hist_get(ile_ctx *c, int32_t nb, double *P_ra, double *P_sd)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (!P_ra || !P_sd) return fail(c, ILE_E_ARG, "null pointer");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    ile_status s = hist_init(c, nb, false);
    if (s) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(P_ra, c->hP.p, nb * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(P_sd, (double *)c->hP.p + nb, nb * sizeof(double),
                         hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_hist_set(ile_ctx *c, int32_t nb, const double *P_ra, const double *P_sd)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (!P_ra || !P_sd) return fail(c, ILE_E_ARG, "null pointer");
    double sr = 0, ss = 0;
    for (int b = 0; b < nb; b++) {
        if (!(P_ra[b] > 0) || !(P_sd[b] > 0) || !std::isfinite(P_ra[b]) ||
            !std::isfinite(P_sd[b]))
            return fail(c, ILE_E_ARG, "histogram bin %d not positive and finite", b);
        sr += P_ra[b];
        ss += P_sd[b];
    }
    if (std::fabs(sr - 1) > 1e-9 || std::fabs(ss - 1) > 1e-9)
        return fail(c, ILE_E_ARG, "histograms must sum to 1");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    ile_status s = hist_init(c, nb, true);
    if (s) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->hP.p, P_ra, nb * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((double *)c->hP.p + nb, P_sd, nb * sizeof(double),
                         hipMemcpyHostToDevice));
    // the cumulative sums follow the bins' order
    HIP_TRY(c, ile_launch_hist_cdf(nb, (const double *)c->hP.p, (double *)c->hC.p,
                                   c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ILE_OK;
}

ile_status ile_hist_draw_dev(ile_ctx *c, uint64_t seed, int64_t first, int64_t N,
                             double d_min, double d_max, double *smp, int64_t ld,
                             double *lp, double *lq, int32_t *bins)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (N < 0 || first < 0 || (N > 0 && !smp) || ld < N || !(d_min > 0) ||
        !(d_max > d_min) || !std::isfinite(d_max))
        return fail(c, ILE_E_ARG, "bad draw arguments");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    ile_status s = hist_init(c, c->hist_nb ? c->hist_nb : 50, false);
    if (s) return s;
    HIP_TRY(c, ile_launch_hist_draw(seed, first, N, c->hist_nb, (const double *)c->hP.p,
                                    (const double *)c->hC.p, d_min, d_max,
                                    c->cfg.t_ref_max_s, smp, ld, lp, lq, bins, c->stream));
    return ILE_OK;
}

static ile_status refit_impl(ile_ctx *c, const int32_t *bins, int64_t ld, const double *lnL,
                             const double *lp, const double *lq, int64_t N, double floor_w,
                             double temper)
{
    ile_status s;
    if ((s = ensure(c, c->hist_tmp, ile_hist_refit_tmp_doubles(N, c->hist_nb) * sizeof(double))))
        return s;
    HIP_TRY(c, ile_launch_hist_refit(bins, ld, lnL, lp, lq, N, c->hist_nb, floor_w, temper,
                                     (double *)c->hist_tmp.p, (double *)c->hP.p,
                                     (double *)c->hC.p, c->stream));
    return ILE_OK;
}

ile_status ile_hist_refit_dev(ile_ctx *c, const int32_t *bins, int64_t ld, const double *lnL,
                              const double *lp, const double *lq, int64_t N, double floor_w,
                              double temper)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    if (N <= 0 || !bins || !lnL || ld < N || !(floor_w >= 0 && floor_w <= 1) || !(temper > 0))
        return fail(c, ILE_E_ARG, "bad refit arguments");
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    ile_status s = hist_init(c, c->hist_nb ? c->hist_nb : 50, false);
    if (s) return s;
    return refit_impl(c, bins, ld, lnL, lp, lq, N, floor_w, temper);
}

// Sampler LEARNED: adaptive rounds (training set), training, then chunks
// from the defensive mixture; falls back to the adaptive sampler if the
// first learned chunk's n_eff is below the threshold.
static ile_status run_learned(ile_ctx *c, const ile_run_opts *o, ile_result *out,
                              int64_t *n_chunks_out)
{
    ile_status s;
    if (!o->prop) return fail(c, ILE_E_ARG, "sampler LEARNED needs a proposal");
    if (ile_prop_stream(o->prop) != c->stream)
        return fail(c, ILE_E_ARG, "the proposal must use the context's stream");
    if (o->max_samples <= 0 || !(o->d_min_mpc > 0) || !(o->d_max_mpc > o->d_min_mpc) ||
        !std::isfinite(o->d_max_mpc))
        return fail(c, ILE_E_ARG, "bad run options");
    const int64_t chunk = o->chunk > 0 ? o->chunk : 100000;
    const int rounds = o->adapt_chunks > 0 ? o->adapt_chunks : 3;
    const int nb = o->n_bins > 0 ? o->n_bins : 50;
    const double floor_w = o->floor >= 0 ? o->floor : 0.1;
    const double temper = o->temper > 0 ? o->temper : 10.0;
    const double eps = o->eps >= 0 ? o->eps : 0.1;
    const double fb = o->fallback_neff >= 0 ? o->fallback_neff : 1000.0;
    const int refine_rounds = o->refine_rounds >= 0 ? o->refine_rounds : 24;
    const int refine_steps = o->refine_steps > 0 ? o->refine_steps : 150;
    const double refine_eff = o->refine_eff > 0 ? o->refine_eff : 0.05;
    const double kappa = o->sigma_scale > 0 ? o->sigma_scale : 1.2;
    if (floor_w > 1 || eps >= 1) return fail(c, ILE_E_ARG, "floor > 1 or eps >= 1");
    if (!std::isfinite(kappa)) return fail(c, ILE_E_ARG, "bad sigma scale");
    if (ile_prop_set_sigma_scale(o->prop, kappa) != ILE_OK)
        return fail(c, ILE_E_DEVICE, "sigma scale: %s", ile_prop_last_error(o->prop));
    const int64_t ntr = (int64_t)rounds * chunk;
    if (ntr > ((int64_t)1 << 30)) return fail(c, ILE_E_ARG, "training set too large");
    const int64_t max_chunks = (o->max_samples + chunk - 1) / chunk;
    if (max_chunks > (1 << 22)) return fail(c, ILE_E_ARG, "too many chunks");
    if ((s = hist_init(c, nb, o->reset != 0))) return s;
    if ((s = ensure(c, c->smp, (size_t)chunk * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->out, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnp, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnq, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->bins, (size_t)chunk * 2 * sizeof(int32_t)))) return s;
    // one extra partial slot for the refinement chunks' own n_eff
    if ((s = ensure(c, c->parts, (size_t)(max_chunks + 1) * 5 * sizeof(double)))) return s;
    if ((s = ensure(c, c->trx, (size_t)ntr * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->trw, (size_t)ntr * sizeof(double)))) return s;
    if ((s = ensure_work(c, chunk))) return s;
    c->learned = ile_learned_info{};
    double *smp = (double *)c->smp.p, *lp = (double *)c->lnp.p, *lq = (double *)c->lnq.p;
    double *trx = (double *)c->trx.p, *trw = (double *)c->trw.p;
    const ile_mdn_mix mix{nb, (const double *)c->hP.p, (const double *)c->hC.p, eps};
    const bool warm = o->warm != 0;
    // 1. adaptive rounds: the training set, drawn from the histograms (refit
    //    after each round), or from the carried-over mixture when warm
    for (int rd = 0; rd < rounds; rd++) {
        const int64_t first = (int64_t)rd * chunk;
        if (warm)
            HIP_TRY(c, ile_launch_mdn_sample(ile_prop_dev(o->prop), mix, o->seed, first, chunk,
                                             smp, chunk, lp, lq, ile_prop_grid(o->prop),
                                             c->stream));
        else
            HIP_TRY(c, ile_launch_hist_draw(o->seed, first, chunk, nb, (const double *)c->hP.p,
                                            (const double *)c->hC.p, o->d_min_mpc, o->d_max_mpc,
                                            c->cfg.t_ref_max_s, smp, chunk, lp, lq,
                                            (int32_t *)c->bins.p, c->stream));
        if ((s = run_eval(c, smp, chunk, (double *)c->out.p, nullptr))) return s;
        HIP_TRY(c, hipMemcpy2DAsync(trx + first, (size_t)ntr * sizeof(double), smp,
                                    (size_t)chunk * sizeof(double), (size_t)chunk * sizeof(double),
                                    7, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, ile_launch_lnw((const double *)c->out.p, lp, lq, chunk, trw + first,
                                  c->stream));
        if (!warm && (s = refit_impl(c, (const int32_t *)c->bins.p, chunk,
                                     (const double *)c->out.p, lp, lq, chunk, floor_w, temper)))
            return s;
    }
    // 2. training
    ile_prop_train_opts to{};
    to.steps = warm ? refine_steps : (o->train_steps > 0 ? o->train_steps : 300);
    to.batch = o->train_batch > 0 ? o->train_batch : 16384;
    to.lr = o->lr > 0 ? o->lr : 2e-3;
    to.ess_frac = o->train_ess > 0 ? o->train_ess : 0.01;
    to.seed = o->seed;
    to.fit_transform = 1;
    double loss = 0.0;
    if (ile_prop_train_dev(o->prop, trx, ntr, trw, ntr, &to, &loss) != ILE_OK)
        return fail(c, ILE_E_DEVICE, "training failed: %s", ile_prop_last_error(o->prop));
    c->learned.n_train_samples = ntr;
    c->learned.train_ms = ile_prop_last_ms(o->prop);
    c->learned.final_loss = loss;
    double r[6] = {0, 0, 0, 0, 0, 0};
    // 3. refinement: each chunk of the mixture replaces the oldest chunk of
    //    the training ring and the network is refit, until a chunk is
    //    efficient enough or the rounds run out.  Then a probe chunk of the
    //    current mixture, never part of the estimate: if its n_eff is below
    //    fallback_neff it becomes one more refinement chunk while rounds
    //    remain, else the run falls back to the adaptive sampler.
    double *rpart = (double *)c->parts.p + 5 * max_chunks;
    int64_t first0 = ntr;
    to.steps = refine_steps;
    int rr = 0, rec = 0;
    bool learned = true;
    // one chunk of the current mixture: draw, evaluate, its own n_eff in r
    auto mixture_chunk = [&](double *r) -> ile_status {
        ile_status s2;
        HIP_TRY(c, ile_launch_mdn_sample(ile_prop_dev(o->prop), mix, o->seed, first0, chunk, smp,
                                         chunk, lp, lq, ile_prop_grid(o->prop), c->stream));
        first0 += chunk;
        if ((s2 = run_eval(c, smp, chunk, (double *)c->out.p, nullptr))) return s2;
        HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, lp, lq, chunk,
                                     (double *)c->red_tmp.p, rpart, c->stream));
        HIP_TRY(c, ile_launch_finish(rpart, 1, (double *)c->res.p, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(r, c->res.p, 6 * sizeof(double), hipMemcpyDeviceToHost));
        c->learned.n_refine_samples += chunk;
        c->learned.last_refine_eff = r[1] / (double)chunk;
        if (rec < 32) {
            c->learned.refine_eff[rec] = c->learned.last_refine_eff;
            c->learned.refine_kish[rec] = r[2] / (double)chunk;
        }
        rec++;
        return ILE_OK;
    };
    // the last chunk into the ring (slot of refinement round rr), then refit
    auto refit_with_chunk = [&]() -> ile_status {
        const int64_t slot = (int64_t)(rr % rounds) * chunk;
        rr++;
        HIP_TRY(c, hipMemcpy2DAsync(trx + slot, (size_t)ntr * sizeof(double), smp,
                                    (size_t)chunk * sizeof(double), (size_t)chunk * sizeof(double),
                                    7, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, ile_launch_lnw((const double *)c->out.p, lp, lq, chunk, trw + slot, c->stream));
        if (ile_prop_train_dev(o->prop, trx, ntr, trw, ntr, &to, &loss) != ILE_OK)
            return fail(c, ILE_E_DEVICE, "refit failed: %s", ile_prop_last_error(o->prop));
        c->learned.train_ms += ile_prop_last_ms(o->prop);
        c->learned.final_loss = loss;
        return ILE_OK;
    };
    for (;;) {
        while (rr < refine_rounds) {
            if ((s = mixture_chunk(r))) return s;
            if (r[1] >= refine_eff * (double)chunk) break;
            if (o->refine_kish > 0 && r[2] >= o->refine_kish * (double)chunk) break;
            if ((s = refit_with_chunk())) return s;
        }
        if (fb <= 0) break;
        if ((s = mixture_chunk(r))) return s;   // the probe
        if (r[1] >= fb) break;
        if (rr >= refine_rounds) {
            learned = false;
            c->learned.fell_back = 1;
            break;
        }
        if ((s = refit_with_chunk())) return s;
    }
    // 4. estimation chunks from the defensive mixture, or from the adaptive
    //    sampler after a fallback
    int64_t done = 0, ci = 0;
    while (done < o->max_samples) {
        const int64_t n = std::min(chunk, o->max_samples - done);
        const int64_t first = first0 + done;
        if (learned) {
            HIP_TRY(c, ile_launch_mdn_sample(ile_prop_dev(o->prop), mix, o->seed, first, n, smp,
                                             n, lp, lq, ile_prop_grid(o->prop), c->stream));
        } else {
            HIP_TRY(c, ile_launch_hist_draw(o->seed, first, n, nb, (const double *)c->hP.p,
                                            (const double *)c->hC.p, o->d_min_mpc,
                                            o->d_max_mpc, c->cfg.t_ref_max_s, smp, n, lp, lq,
                                            (int32_t *)c->bins.p, c->stream));
        }
        if ((s = run_eval(c, smp, n, (double *)c->out.p, nullptr))) return s;
        HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, lp, lq, n,
                                     (double *)c->red_tmp.p, (double *)c->parts.p + 5 * ci,
                                     c->stream));
        if (!learned && (s = refit_impl(c, (const int32_t *)c->bins.p, n, (const double *)c->out.p,
                                        lp, lq, n, floor_w, temper)))
            return s;
        HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, (int)(ci + 1),
                                     (double *)c->res.p, c->stream));
        done += n;
        ci++;
        if (learned) c->learned.n_learned_samples += n;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(r, c->res.p, sizeof(r), hipMemcpyDeviceToHost));
        if (o->n_eff_target > 0 && r[1] >= o->n_eff_target) break;
    }
    if ((s = finish_call(c))) return s;
    fetched_result(c, r);
    copy_result(r, out);
    if (n_chunks_out) *n_chunks_out = ci;
    return ILE_OK;
}

ile_status ile_last_learned_info(const ile_ctx *c, ile_learned_info *out)
{
    if (!c || !out) return ILE_E_ARG;
    *out = c->learned;
    return ILE_OK;
}

ile_status ile_run(ile_ctx *c, const ile_run_opts *o, ile_result *out, int64_t *n_chunks_out)
{
    ile_status s = check_ready(c);
    if (s) return s;
    if (!o || !out) return fail(c, ILE_E_ARG, "null pointer");
    const int32_t sampler = enum_raw(o->sampler);
    if (sampler == ILE_SAMPLER_LEARNED) return run_learned(c, o, out, n_chunks_out);
    if (sampler != ILE_SAMPLER_PRIOR && sampler != ILE_SAMPLER_ADAPTIVE)
        return fail(c, ILE_E_ARG, "unknown sampler");
    if (o->max_samples <= 0 || !(o->d_min_mpc > 0) || !(o->d_max_mpc > o->d_min_mpc) ||
        !std::isfinite(o->d_max_mpc))
        return fail(c, ILE_E_ARG, "bad run options");
    const int64_t chunk = std::min<int64_t>(o->chunk > 0 ? o->chunk : 100000, o->max_samples);
    const int nb = o->n_bins > 0 ? o->n_bins : 50;
    const double floor_w = o->floor >= 0 ? o->floor : 0.1;
    const double temper = o->temper > 0 ? o->temper : 10.0;
    if (floor_w > 1) return fail(c, ILE_E_ARG, "floor > 1");
    const bool adaptive = o->sampler == ILE_SAMPLER_ADAPTIVE;
    const int64_t max_chunks = (o->max_samples + chunk - 1) / chunk;
    if (max_chunks > (1 << 22)) return fail(c, ILE_E_ARG, "too many chunks");
    if (adaptive && (s = hist_init(c, nb, o->reset != 0))) return s;
    if ((s = ensure(c, c->smp, (size_t)chunk * 7 * sizeof(double)))) return s;
    if ((s = ensure(c, c->out, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnp, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->lnq, (size_t)chunk * sizeof(double)))) return s;
    if ((s = ensure(c, c->bins, (size_t)chunk * 2 * sizeof(int32_t)))) return s;
    if ((s = ensure(c, c->parts, (size_t)max_chunks * 5 * sizeof(double)))) return s;
    if ((s = ensure_work(c, chunk))) return s;
    bool adapting = adaptive;
    int64_t done = 0, ci = 0;
    double r[6] = {0, 0, 0, 0, 0, 0};
    while (done < o->max_samples) {
        const int64_t n = std::min(chunk, o->max_samples - done);
        double *smp = (double *)c->smp.p, *lp = nullptr, *lq = nullptr;
        if (adaptive) {
            lp = (double *)c->lnp.p;
            lq = (double *)c->lnq.p;
            HIP_TRY(c, ile_launch_hist_draw(o->seed, done, n, nb, (const double *)c->hP.p,
                                            (const double *)c->hC.p, o->d_min_mpc,
                                            o->d_max_mpc, c->cfg.t_ref_max_s, smp, n, lp, lq,
                                            (int32_t *)c->bins.p, c->stream));
        } else {
            HIP_TRY(c, ile_launch_prior(o->seed, done, n, o->d_min_mpc, o->d_max_mpc,
                                        c->cfg.t_ref_max_s, smp, n, nullptr, c->stream));
        }
        if ((s = run_eval(c, smp, n, (double *)c->out.p, nullptr))) return s;
        HIP_TRY(c, ile_launch_reduce((const double *)c->out.p, lp, lq, n,
                                     (double *)c->red_tmp.p, (double *)c->parts.p + 5 * ci,
                                     c->stream));
        if (adapting &&
            (s = refit_impl(c, (const int32_t *)c->bins.p, n, (const double *)c->out.p, lp,
                            lq, n, floor_w, temper)))
            return s;
        HIP_TRY(c, ile_launch_finish((const double *)c->parts.p, (int)(ci + 1),
                                     (double *)c->res.p, c->stream));
        done += n;
        ci++;
        const bool check = o->n_eff_target > 0 || (adapting && o->adapt_chunks < 0);
        if (check || done >= o->max_samples) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipMemcpy(r, c->res.p, sizeof(r), hipMemcpyDeviceToHost));
            if (o->n_eff_target > 0 && r[1] >= o->n_eff_target) break;
            if (adapting && o->adapt_chunks < 0 && r[0] > std::max(10.0, 0.5 * r[4]))
                adapting = false;
        }
        if (adapting && o->adapt_chunks >= 0 && ci >= o->adapt_chunks) adapting = false;
    }
    if ((s = finish_call(c))) return s;
    fetched_result(c, r);
    copy_result(r, out);
    if (n_chunks_out) *n_chunks_out = ci;
    return ILE_OK;
}

ile_status ile_get_stream(const ile_ctx *c, void **stream_out)
{
    if (!c || !stream_out) return ILE_E_ARG;
    *stream_out = (void *)c->stream;
    return ILE_OK;
}

ile_status ile_sync(ile_ctx *c)
{
    if (!c) return ILE_E_ARG;
    ile_status s = finish_call(c);
    c->n_ev_used = 0;
    return s;
}

ile_status ile_set_option(ile_ctx *c, ile_option opt, int64_t v)
{
    if (!c) return ILE_E_ARG;
    begin_call(c);
    ile_tune t = c->tune;
    switch (enum_raw(opt)) {
    case ILE_OPT_SORT:
        if (v != 0 && v != 1) return fail(c, ILE_E_ARG, "sort must be 0 or 1");
        c->sort = (int)v;
        return ILE_OK;
    case ILE_OPT_ENGINE:
        if (v < 0 || v > 2) return fail(c, ILE_E_ARG, "engine must be 0, 1 or 2");
        // option 1 is the phased matrix-core engine where the precision has
        // one (FP64, FP32), else the pipelined one; option 2 the pipelined
        t.engine = v == 0 ? 0 : (v == 1 && c->cfg.precision != ILE_BF16) ? 3 : 1;
        // the vector engine has no 128/192-position blocks: use 256; the
        // phased engine takes 256 or 512 threads (512 by default), the
        // pipelined one 128 positions by default
        if (t.engine == 0 && (t.threads == 128 || t.threads == 192)) t.threads = 256;
        if (t.engine == 3 && t.threads != 256) t.threads = 512;
        if (t.engine == 1 && c->tune.engine == 3) t.threads = 128;
        break;
    case ILE_OPT_THREADS:
        t.threads = (int)v;
        break;
    case ILE_OPT_LDS_KB:
        if (v < 0 || v > 160) return fail(c, ILE_E_ARG, "LDS budget must be 0 .. 160 KB");
        t.lds_budget = (int)v * 1024;
        break;
    case ILE_OPT_HARVEST_ROWS:
        if (v < 0) return fail(c, ILE_E_ARG, "harvest rows must be >= 0");
        c->hv_rows = v;
        return ILE_OK;
    default:
        return fail(c, ILE_E_ARG, "unknown option %d", (int)opt);
    }
    if (!ile_tune_supported(c->cfg.precision, t))
        return fail(c, ILE_E_UNSUPPORTED, "tuning not supported for this precision");
    c->tune = t;
    return ILE_OK;
}

double ile_last_kernel_ms(const ile_ctx *c) { return c ? c->last_ms : 0.0; }

void ile_destroy(ile_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (DevBuf *b : {&c->Q, &c->U, &c->V, &c->smp, &c->out, &c->lnp, &c->lnq,
                      &c->shifts, &c->keys, &c->perm, &c->hist, &c->scan_tmp,
                      &c->errflag, &c->red_tmp, &c->parts, &c->res, &c->series,
                      &c->hP, &c->hC, &c->bins, &c->hist_tmp, &c->trx, &c->trw,
                      &c->hv_w, &c->hv_cdf, &c->hv_ws, &c->hv_part, &c->hv_flag, &c->hv_sel,
                      &c->fd_tmp, &c->fd_flag, &c->fd_in, &c->fd_out, &c->rom_A, &c->rom_Z,
                      &c->uvt, &c->terms, &c->smp_s, &c->sh_s})
        release(*b);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    if (c->hpin) (void)hipHostFree(c->hpin);
    delete c;
}

}  // extern "C"
