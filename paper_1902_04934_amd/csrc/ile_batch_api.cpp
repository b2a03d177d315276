// ile_batch_api.cpp -- host side of the batched form (include/ile.h):
// per-point contexts (validation, geometry and device copies reuse the
// single-point code), the concatenated work buffers, the (point, tile)
// queue, the HIP graph of one run, and the autotuner with its text cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ile.h"
#include "ile_internal.h"

const ile_geom &ile_ctx_geom(const ile_ctx *c);
const void *ile_ctx_Q(const ile_ctx *c);
const double *ile_ctx_U(const ile_ctx *c);
const double *ile_ctx_V(const ile_ctx *c);
const double *ile_ctx_uvt(const ile_ctx *c);

namespace {

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

constexpr int kKeyBits = 15;   // ordering key bits per point (buckets 2^15 + 1)
// Largest per-sample terms buffer of one batched run (the phased engine);
// a run that needs more forms the terms in its tiles.
constexpr size_t kMaxTermsBytes = (size_t)32 << 30;

}  // namespace

struct ile_batch {
    ile_batch_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<ile_ctx *> pts;
    ile_batch_tuning tune{256, 2, 0, 1};
    int cu_count = 0, lds_max = 0;
    std::string dev_name;
    Buf geoms, pdev, items, offs, seed, counter, smp, out, shifts, keys, perm, hist, scan_tmp,
        errflag, res, lw, terms;
    // graph of one run and what it was built for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t g_n = -1;
    int g_ext = -1;   // 1: the graph evaluates caller-supplied draws
    double g_dmin = 0, g_dmax = 0;
    ile_batch_tuning g_tune{0, 0, 0, 0};
    size_t g_points = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double last_ms = 0.0;
};

namespace {

ile_status bfail(ile_batch *b, ile_status s, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return s;
}

#define BHIP(b, expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bfail((b), e_ == hipErrorOutOfMemory ? ILE_E_NOMEM : ILE_E_DEVICE,       \
                         "%s: %s", #expr, hipGetErrorString(e_));                           \
    } while (0)

ile_status bensure(ile_batch *b, Buf &x, size_t bytes)
{
    if (x.p && x.bytes >= bytes) return ILE_OK;
    if (x.p) {
        BHIP(b, hipStreamSynchronize(b->stream));
        (void)hipFree(x.p);
        x.p = nullptr;
        x.bytes = 0;
    }
    const size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&x.p, want);
    if (e != hipSuccess) {
        x.p = nullptr;
        return bfail(b, ILE_E_NOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
    }
    x.bytes = want;
    return ILE_OK;
}

void drop_graph(ile_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_n = -1;
}

// The per-point tuning of a batch tuning: engine 1 is the phased matrix-core
// engine for FP64 and FP32 (threads = workgroup size) and the pipelined one
// for BF16; engine 2 the pipelined one (threads = positions per block).
ile_tune point_tune(ile_precision prec, const ile_batch_tuning &bt)
{
    const int eng = bt.engine == 0 ? 0 : (bt.engine == 1 && prec != ILE_BF16) ? 3 : 1;
    ile_tune t{16, bt.threads, eng, 0};
    return t;
}
ile_tune point_tune(const ile_batch *b) { return point_tune(b->cfg.precision, b->tune); }

// the per-point geometry with the batch's 15-bit ordering key
ile_geom batched_geom(const ile_ctx *c)
{
    ile_geom g = ile_ctx_geom(c);
    const int dims = g.key_dims;
    const int bits = kKeyBits / dims;
    int shift = g.key_shift;
    const int64_t width = ((int64_t)1 << (g.key_bits + g.key_shift));
    while ((width >> shift) > ((int64_t)1 << bits)) shift++;
    g.key_shift = shift;
    g.key_bits = bits;
    return g;
}

// Build buffers, queue and the graph of one run for n samples per point:
// prior draws (ext = false) or draws the caller copied to smp with their
// ln p - ln q in lw (ext = true).
ile_status build(ile_batch *b, int64_t n, double dmin, double dmax, bool ext)
{
    drop_graph(b);
    const int P = (int)b->pts.size();
    const int64_t NT = n * P;
    if (NT > 0x7fffffff) return bfail(b, ILE_E_ARG, "too many samples in one batch run");
    const uint32_t B = (1u << kKeyBits) + 1u;
    const int64_t nb = (int64_t)P * B;
    if (ile_scan_tmp_words(nb) > 4096)
        return bfail(b, ILE_E_UNSUPPORTED, "too many points for one sort (%d)", P);
    const ile_tune tu = point_tune(b);
    if (!ile_tune_supported(b->cfg.precision, tu))
        return bfail(b, ILE_E_UNSUPPORTED, "tuning not supported for this precision");
    std::vector<ile_geom> gs(P);
    std::vector<ile_point_dev> pd(P);
    std::vector<int64_t> offs(P + 1);
    size_t dyn = 0, lds = 0;
    for (int p = 0; p < P; p++) {
        gs[p] = batched_geom(b->pts[p]);
        ile_contract_prepare(gs[p], b->cfg.precision, tu);
        offs[p] = (int64_t)p * n;
        dyn = std::max(dyn, ile_contract_dyn_bytes(gs[p], b->cfg.precision, tu));
        lds = std::max(lds, ile_contract_lds_bytes(gs[p], b->cfg.precision, tu));
    }
    offs[P] = NT;
    if (lds > (size_t)b->lds_max)
        return bfail(b, ILE_E_UNSUPPORTED, "needs %zu bytes of LDS per workgroup", lds);
    ile_status s;
    if ((s = bensure(b, b->geoms, P * sizeof(ile_geom)))) return s;
    if ((s = bensure(b, b->pdev, P * sizeof(ile_point_dev)))) return s;
    if ((s = bensure(b, b->offs, (P + 1) * sizeof(int64_t)))) return s;
    if ((s = bensure(b, b->seed, 16))) return s;
    if ((s = bensure(b, b->counter, 16))) return s;
    if ((s = bensure(b, b->smp, (size_t)NT * 7 * sizeof(double)))) return s;
    if ((s = bensure(b, b->out, (size_t)NT * sizeof(double)))) return s;
    if ((s = bensure(b, b->shifts, (size_t)NT * ILE_MAX_DET * sizeof(int32_t)))) return s;
    if ((s = bensure(b, b->keys, (size_t)NT * sizeof(uint32_t)))) return s;
    if ((s = bensure(b, b->perm, (size_t)NT * sizeof(int32_t)))) return s;
    if ((s = bensure(b, b->hist, (size_t)nb * sizeof(uint32_t)))) return s;
    if ((s = bensure(b, b->scan_tmp, (size_t)ile_scan_tmp_words(nb) * 4 + 16))) return s;
    if ((s = bensure(b, b->errflag, 16))) return s;
    if ((s = bensure(b, b->res, (size_t)P * 6 * sizeof(double)))) return s;
    if (ext && (s = bensure(b, b->lw, (size_t)NT * sizeof(double)))) return s;
    // the phased engine's per-sample terms, per point, when they fit in
    // kMaxTermsBytes (else the tiles form them)
    std::vector<size_t> toff(P + 1, 0);
    const bool ph = ile_contract_uses_terms(b->cfg.precision, tu);
    for (int p = 0; p < P; p++)
        toff[p + 1] = toff[p] + (size_t)ile_terms_fields(gs[p]) * (size_t)((n + 15) & ~15);
    const bool use_terms = ph && toff[P] * sizeof(double) <= kMaxTermsBytes;
    if (use_terms && (s = bensure(b, b->terms, toff[P] * sizeof(double)))) return s;
    double *smp = (double *)b->smp.p, *out = (double *)b->out.p;
    int32_t *sh = (int32_t *)b->shifts.p, *perm = (int32_t *)b->perm.p;
    for (int p = 0; p < P; p++) {
        pd[p].Q = ile_ctx_Q(b->pts[p]);
        pd[p].U = (const double2 *)ile_ctx_U(b->pts[p]);
        pd[p].V = (const double2 *)ile_ctx_V(b->pts[p]);
        pd[p].smp = smp + 7 * offs[p];
        pd[p].N = n;
        pd[p].perm = perm + offs[p];
        pd[p].shifts = sh + (int64_t)ILE_MAX_DET * offs[p];
        pd[p].out = out + offs[p];
        pd[p].terms = use_terms ? (const double *)b->terms.p + toff[p] : nullptr;
    }
    // queue: tiles of every point; order 0 = decreasing per-tile cost
    std::vector<int> order(P);
    for (int p = 0; p < P; p++) order[p] = p;
    if (b->tune.order == 0)
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const double cx = (double)gs[x].n_det * gs[x].n_lm * gs[x].n_t;
            const double cy = (double)gs[y].n_det * gs[y].n_lm * gs[y].n_t;
            return cx > cy;
        });
    const int64_t tiles = (n + 15) / 16;
    std::vector<int2> items;
    items.reserve((size_t)tiles * P);
    for (int p : order)
        for (int64_t t = 0; t < tiles; t++) items.push_back(make_int2(p, (int)t));
    if ((s = bensure(b, b->items, items.size() * sizeof(int2)))) return s;
    BHIP(b, hipMemcpy(b->geoms.p, gs.data(), P * sizeof(ile_geom), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->pdev.p, pd.data(), P * sizeof(ile_point_dev), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->offs.p, offs.data(), (P + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->items.p, items.data(), items.size() * sizeof(int2),
                      hipMemcpyHostToDevice));
    BHIP(b, hipMemset(b->errflag.p, 0, 16));
    // all points share one t_ref bound in the draw: the smallest
    double tmax = 1e300;
    for (int p = 0; p < P; p++) tmax = std::min(tmax, gs[p].t_ref_max);

    hipStream_t st = b->stream;
    BHIP(b, ile_contract_batched_allow(b->cfg.precision, tu, dyn));
    BHIP(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int grid = b->cu_count * b->tune.wgs_per_cu;
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    step(ile_launch_fill_u32((uint32_t *)b->counter.p, 0u, 1, st));
    step(ile_launch_fill_u32((uint32_t *)b->hist.p, 0u, nb, st));
    if (!ext)
        step(ile_launch_prior_multi((const uint64_t *)b->seed.p, (const int64_t *)b->offs.p, P,
                                    NT, dmin, dmax, tmax, smp, st));
    step(ile_launch_prep_multi((const ile_geom *)b->geoms.p, (const int64_t *)b->offs.p, P, NT,
                               smp, sh, (uint32_t *)b->keys.p, (uint32_t *)b->hist.p, B,
                               (int32_t *)b->errflag.p, st));
    step(ile_launch_scan((uint32_t *)b->hist.p, nb, (uint32_t *)b->scan_tmp.p, st));
    step(ile_launch_scatter_multi((const uint32_t *)b->keys.p, (const int64_t *)b->offs.p, P,
                                  NT, (uint32_t *)b->hist.p, perm, st));
    if (use_terms)
        for (int p = 0; p < P; p++)
            step(ile_launch_terms(gs[p], pd[p].smp, n, pd[p].perm, pd[p].shifts,
                                  ile_ctx_uvt(b->pts[p]), (double *)pd[p].terms, st));
    step(ile_launch_contract_batched(b->cfg.precision, tu, (const ile_geom *)b->geoms.p,
                                     (const ile_point_dev *)b->pdev.p,
                                     (const int2 *)b->items.p, (int)items.size(),
                                     (unsigned *)b->counter.p, grid, dyn, use_terms, st));
    step(ile_launch_reduce_points(out, ext ? (const double *)b->lw.p : nullptr,
                                  (const int64_t *)b->offs.p, P, (double *)b->res.p, st));
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, ILE_E_DEVICE, "graph capture failed: %s",
                     hipGetErrorString(e != hipSuccess ? e : ec));
    }
    b->graph = g;
    BHIP(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->g_n = n;
    b->g_ext = ext ? 1 : 0;
    b->g_dmin = dmin;
    b->g_dmax = dmax;
    b->g_tune = b->tune;
    b->g_points = b->pts.size();
    return ILE_OK;
}

bool same_tune(const ile_batch_tuning &a, const ile_batch_tuning &c)
{
    return a.threads == c.threads && a.wgs_per_cu == c.wgs_per_cu && a.order == c.order &&
           a.engine == c.engine;
}

// (Re)build the graph if the run's shape changed.
ile_status ensure_graph(ile_batch *b, int64_t n, double dmin, double dmax, bool ext)
{
    if (b->g_n != n || b->g_ext != (ext ? 1 : 0) || b->g_dmin != dmin || b->g_dmax != dmax ||
        !same_tune(b->g_tune, b->tune) || b->g_points != b->pts.size() || !b->exec)
        return build(b, n, dmin, dmax, ext);
    return ILE_OK;
}

ile_status run_graph(ile_batch *b, uint64_t seed, int64_t n, double dmin, double dmax,
                     bool ext = false)
{
    ile_status s;
    if ((s = ensure_graph(b, n, dmin, dmax, ext))) return s;
    BHIP(b, hipMemcpyAsync(b->seed.p, &seed, sizeof(seed), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipEventRecord(b->e0, b->stream));
    BHIP(b, hipGraphLaunch(b->exec, b->stream));
    BHIP(b, hipEventRecord(b->e1, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, b->e0, b->e1));
    b->last_ms = ms;
    int32_t flag = 0;
    BHIP(b, hipMemcpy(&flag, b->errflag.p, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag) {
        BHIP(b, hipMemset(b->errflag.p, 0, 16));
        if (flag & 2) return bfail(b, ILE_E_RANGE, "invalid ln_p/ln_q of a draw");
        return bfail(b, ILE_E_RANGE,
                     "a sample is outside the prior support or its window left its Q");
    }
    return ILE_OK;
}

ile_status copy_results(ile_batch *b, ile_result *results)
{
    const size_t P = b->pts.size();
    std::vector<double> r(6 * P);
    BHIP(b, hipMemcpy(r.data(), b->res.p, r.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t p = 0; p < P; p++) {
        results[p].ln_L_marg = r[6 * p];
        results[p].n_eff = r[6 * p + 1];
        results[p].n_eff_kish = r[6 * p + 2];
        results[p].sigma_ln_L = r[6 * p + 3];
        results[p].max_ln_L = r[6 * p + 4];
        results[p].n_samples = (int64_t)r[6 * p + 5];
    }
    return ILE_OK;
}

std::string signature(const ile_batch *b, int64_t n)
{
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the points' shapes
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; i++) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const ile_ctx *c : b->pts) {
        const ile_geom &g = ile_ctx_geom(c);
        mix(g.n_det);
        mix(g.n_lm);
        mix(g.n_t);
        mix(g.n_q);
    }
    mix(n);
    std::ostringstream o;
    std::string dn = b->dev_name;
    for (char &ch : dn)
        if (ch == ' ') ch = '_';
    o << dn << "|p" << (int)b->cfg.precision << "|n" << b->pts.size() << "|" << std::hex << h;
    return o.str();
}

}  // namespace

extern "C" {

ile_status ile_batch_create(const ile_batch_config *cfg, ile_batch **out)
{
    if (!out) return ILE_E_ARG;
    *out = nullptr;
    if (!cfg || enum_raw(cfg->precision) < ILE_FP64 || enum_raw(cfg->precision) > ILE_BF16)
        return ILE_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ILE_E_DEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return ILE_E_ARG;
    ile_batch *b = new (std::nothrow) ile_batch();
    if (!b) return ILE_E_NOMEM;
    b->cfg = *cfg;
    hipDeviceProp_t prop;
    if (hipSetDevice(cfg->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) {
        delete b;
        return ILE_E_DEVICE;
    }
    b->cu_count = prop.multiProcessorCount;
    b->lds_max = (int)prop.sharedMemPerBlock;
    b->dev_name = prop.gcnArchName;
    // FP64 and FP32: the phased matrix-core engine in eight-wave
    // workgroups, two per CU (its LDS budget); BF16: the pipelined engine at
    // 128 positions per block, measured fastest on 32 points of the
    // 5-21-mode, 201-1601-bin mix at 1e6 draws each
    b->tune.engine = 1;
    b->tune.threads = cfg->precision == ILE_BF16 ? 128 : 512;
    b->tune.wgs_per_cu = 2;
    if (cfg->stream) {
        b->stream = (hipStream_t)cfg->stream;
    } else if (hipStreamCreate(&b->stream) != hipSuccess) {
        delete b;
        return ILE_E_DEVICE;
    } else {
        b->own_stream = true;
    }
    if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess) {
        ile_batch_destroy(b);
        return ILE_E_DEVICE;
    }
    *out = b;
    return ILE_OK;
}

ile_status ile_batch_add_point(ile_batch *b, const ile_config *pc, const double *Q, int64_t n_q,
                               double t0_s, const double *U, const double *V,
                               const ile_detector *dets, int32_t *id_out)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (!pc) return bfail(b, ILE_E_ARG, "null config");
    ile_config c = *pc;
    c.precision = b->cfg.precision;
    c.device = b->cfg.device;
    c.stream = b->stream;
    ile_ctx *ctx = nullptr;
    ile_status s = ile_create(&c, &ctx);
    if (s) return bfail(b, s, "point %zu: invalid configuration", b->pts.size());
    s = ile_set_data(ctx, Q, n_q, t0_s, U, V, dets);
    if (s) {
        b->err = std::string("point: ") + ile_last_error(ctx);
        ile_destroy(ctx);
        return s;
    }
    b->pts.push_back(ctx);
    drop_graph(b);
    if (id_out) *id_out = (int32_t)b->pts.size() - 1;
    return ILE_OK;
}

int32_t ile_batch_n_points(const ile_batch *b) { return b ? (int32_t)b->pts.size() : 0; }

ile_status ile_batch_run(ile_batch *b, uint64_t seed, int64_t n, double dmin, double dmax,
                         ile_result *results)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (b->pts.empty()) return bfail(b, ILE_E_STATE, "no points");
    if (n <= 0 || !results || !(dmin > 0) || !(dmax > dmin) || !std::isfinite(dmax))
        return bfail(b, ILE_E_ARG, "bad run arguments");
    BHIP(b, hipSetDevice(b->cfg.device));
    ile_status s = run_graph(b, seed, n, dmin, dmax);
    if (s) return s;
    return copy_results(b, results);
}

ile_status ile_batch_run_dev(ile_batch *b, int64_t n, const double *samples_dev,
                             const double *ln_p_dev, const double *ln_q_dev,
                             ile_result *results)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (b->pts.empty()) return bfail(b, ILE_E_STATE, "no points");
    if (n <= 0 || !results || !samples_dev) return bfail(b, ILE_E_ARG, "bad run arguments");
    BHIP(b, hipSetDevice(b->cfg.device));
    ile_status s;
    if ((s = ensure_graph(b, n, 0.0, 0.0, true))) return s;
    const int64_t NT = n * (int64_t)b->pts.size();
    // the caller's [P][7][n] layout is the graph's sample buffer layout
    BHIP(b, hipMemcpyAsync(b->smp.p, samples_dev, (size_t)NT * 7 * sizeof(double),
                           hipMemcpyDeviceToDevice, b->stream));
    BHIP(b, ile_launch_batch_lw(ln_p_dev, ln_q_dev, NT, (double *)b->lw.p,
                                (int32_t *)b->errflag.p, b->stream));
    if ((s = run_graph(b, 0, n, 0.0, 0.0, true))) return s;
    return copy_results(b, results);
}

ile_status ile_batch_lnL(ile_batch *b, double *out, int64_t n_total)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (!out || b->g_n < 0 || n_total != b->g_n * (int64_t)b->g_points)
        return bfail(b, ILE_E_ARG, "n_total must equal points x samples of the last run");
    BHIP(b, hipStreamSynchronize(b->stream));
    BHIP(b, hipMemcpy(out, b->out.p, n_total * sizeof(double), hipMemcpyDeviceToHost));
    return ILE_OK;
}

ile_status ile_batch_set_tuning(ile_batch *b, const ile_batch_tuning *t)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (!t || (t->threads != 128 && t->threads != 192 && t->threads != 256 && t->threads != 512) ||
        t->wgs_per_cu < 1 ||
        t->wgs_per_cu > 4 || (t->order != 0 && t->order != 1) ||
        t->engine < 0 || t->engine > 2)
        return bfail(b, ILE_E_ARG, "bad tuning");
    const ile_tune tu = point_tune(b->cfg.precision, *t);
    if (!ile_tune_supported(b->cfg.precision, tu))
        return bfail(b, ILE_E_UNSUPPORTED, "tuning not supported for this precision");
    // the persistent BF16 kernel of 512-position blocks (1024 threads) is
    // not offered: under the 128-register cap of such workgroups it spills
    // and returned non-finite values (the one-point kernel of that width
    // does not spill and stays available)
    if (b->cfg.precision == ILE_BF16 && tu.engine == 1 && tu.threads == 512)
        return bfail(b, ILE_E_UNSUPPORTED, "BF16 batches take 128 to 256 positions per block");
    b->tune = *t;
    return ILE_OK;
}

ile_status ile_batch_get_tuning(const ile_batch *b, ile_batch_tuning *t)
{
    if (!b || !t) return ILE_E_ARG;
    *t = b->tune;
    return ILE_OK;
}

ile_status ile_batch_autotune(ile_batch *b, int64_t n, const char *cache_path)
{
    if (!b) return ILE_E_ARG;
    b->err.clear();
    if (b->pts.empty()) return bfail(b, ILE_E_STATE, "no points");
    if (n <= 0) return bfail(b, ILE_E_ARG, "bad sample count");
    BHIP(b, hipSetDevice(b->cfg.device));
    const std::string key = signature(b, n);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            ile_batch_tuning t{};
            double ms = 0;
            if ((ls >> k >> t.threads >> t.wgs_per_cu >> t.order >> t.engine >> ms) && k == key &&
                ile_batch_set_tuning(b, &t) == ILE_OK)
                return ILE_OK;
        }
    }
    // candidates: the phased engine (workgroups of 256 or 512 threads), the
    // pipelined and the vector engine (positions per block); tunings a
    // precision does not take are skipped
    std::vector<ile_batch_tuning> cand;
    for (int w : {1, 2, 3})
        for (int o : {0, 1}) {
            for (int th : {256, 512}) cand.push_back({th, w, o, 1});
            for (int th : {128, 192, 256, 512}) cand.push_back({th, w, o, 2});
            for (int th : {256, 512}) cand.push_back({th, w, o, 0});
        }
    ile_batch_tuning best = b->tune;
    double best_ms = 1e300;
    for (const ile_batch_tuning &t : cand) {
        if (ile_batch_set_tuning(b, &t) != ILE_OK) continue;
        ile_status s = run_graph(b, 12345, n, 10.0, 1000.0);   // build + warm
        if (s == ILE_E_UNSUPPORTED) continue;
        if (s) return s;
        if ((s = run_graph(b, 12345, n, 10.0, 1000.0))) return s;
        if (b->last_ms < best_ms) {
            best_ms = b->last_ms;
            best = t;
        }
    }
    b->tune = best;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << " " << best.threads << " " << best.wgs_per_cu << " " << best.order << " "
          << best.engine << " " << best_ms << "\n";
    }
    return ILE_OK;
}

double ile_batch_last_ms(const ile_batch *b) { return b ? b->last_ms : 0.0; }

const char *ile_batch_last_error(const ile_batch *b) { return b ? b->err.c_str() : "null batch"; }

void ile_batch_destroy(ile_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->cfg.device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (ile_ctx *c : b->pts) ile_destroy(c);
    for (Buf *x : {&b->geoms, &b->pdev, &b->items, &b->offs, &b->seed, &b->counter, &b->smp,
                   &b->out, &b->shifts, &b->keys, &b->perm, &b->hist, &b->scan_tmp, &b->errflag,
                   &b->res, &b->lw, &b->terms})
        if (x->p) (void)hipFree(x->p);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
