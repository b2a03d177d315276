// ile_kernels.hip -- gfx950 kernels of the ILE likelihood hot path.
//
// Paper: arXiv:1902.04934.  Sec. II.A defines the per-sample likelihood
// (Eq. (7), matrix form Eq. (10)) and its time marginalization (Eq. (9));
// Sec. II.B describes the GPU step whose most costly part is the contraction
// of Q over detector-dependent time windows; Sec. II.C the Monte Carlo
// accuracy measure.
//
// Pipeline for a block of N samples:
//   k_prep        window starts s_k per (sample, detector), validity,
//                 ordering key (Hilbert index of the window starts)
//   k_scan*       counting sort of the samples by key (cells of nearby windows)
//   k_terms       per sample in tile order: harmonics, antenna factors and the
//                 quadratic term of Eq. (7) (FP64 and FP32 phased engine)
//   k_contract_ph per tile of 16 samples: the coefficients in LDS; per time
//                 chunk and detector the products sum_lm Re(conj(c) Q[p]) over
//                 the union of the tile's windows on the matrix cores (each Q
//                 value loaded once feeds 16 samples), moved to each sample's
//                 bin row and summed over the detectors; FP64 log-sum-exp over
//                 the bins; deterministic tree at the end
//   k_contract    the same with the per-sample work in the tile, producer and
//                 consumer waves (BF16; selectable for FP64/FP32) or VALU
//   k_red*        FP64 importance-sampling partials {M, S1, S2, n, maxL}.
#include <hip/hip_runtime.h>

#include <math.h>

#include <mutex>

#include "ile_internal.h"
#include "ile_rng.h"

namespace {

constexpr double kC = 299792458.0;
constexpr double kTwoPi = 6.283185307179586476925;
constexpr double kPi = 3.141592653589793238463;


// ---------------------------------------------------------------- geometry
// Arrival delay at site k relative to the geocentre, tau = -n.r/c, with n
// the unit vector towards the source (Sec. II.A, detector response).  Same
// operation order as written, no contraction, so that the window rounding
// agrees with an independent evaluation except within 1e-9 of a tie.
__device__ inline double delay_dev(const ile_geom &g, int k, double ra,
                                   double dec)
{
#pragma clang fp contract(off)
    double h = ra - g.gmst;
    double n0 = cos(dec) * cos(h);
    double n1 = cos(dec) * sin(h);
    double n2 = sin(dec);
    double nr = n0 * g.r[k][0] + n1 * g.r[k][1] + n2 * g.r[k][2];
    return -nr / kC;
}

// Antenna patterns from the detector tensor: polarization basis X, Y of a
// source at hour angle h = ra - gmst, declination dec, rotated by psi;
// F+ = X.D.X - Y.D.Y, Fx = X.D.Y + Y.D.X.  tr = (sin h, cos h, sin dec,
// cos dec, sin psi, cos psi).
__device__ inline void antenna_trig(const ile_geom &g, int k, const double tr[6], double &fp,
                                    double &fx)
{
    const double sh = tr[0], ch = tr[1], sd = tr[2], cd = tr[3], sp = tr[4], cp = tr[5];
    const double eE[3] = {-sh, ch, 0.0};
    const double eN[3] = {-sd * ch, -sd * sh, cd};
    double X[3], Y[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        X[i] = -cp * eE[i] + sp * eN[i];
        Y[i] = sp * eE[i] + cp * eN[i];
    }
    double DX[3], DY[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        DX[i] = g.D[k][3 * i] * X[0] + g.D[k][3 * i + 1] * X[1] + g.D[k][3 * i + 2] * X[2];
        DY[i] = g.D[k][3 * i] * Y[0] + g.D[k][3 * i + 1] * Y[1] + g.D[k][3 * i + 2] * Y[2];
    }
    fp = (X[0] * DX[0] + X[1] * DX[1] + X[2] * DX[2]) -
         (Y[0] * DY[0] + Y[1] * DY[1] + Y[2] * DY[2]);
    fx = (X[0] * DY[0] + X[1] * DY[1] + X[2] * DY[2]) +
         (Y[0] * DX[0] + Y[1] * DX[1] + Y[2] * DX[2]);
}

__device__ inline void antenna_dev(const ile_geom &g, int k, double ra,
                                   double dec, double psi, double &fp,
                                   double &fx)
{
    double tr[6];
    sincos(ra - g.gmst, &tr[0], &tr[1]);
    sincos(dec, &tr[2], &tr[3]);
    sincos(psi, &tr[4], &tr[5]);
    antenna_trig(g, k, tr, fp, fx);
}

// Per-sample tables of the tile prologue: the sines and cosines of the
// antenna patterns, powers 0 .. 2 ILE_LMAX of cos(iota/2) and sin(iota/2),
// and e^{i m phi} for |m| <= ILE_LMAX.
constexpr int kPw = 2 * ILE_LMAX + 1;
constexpr int kProTab = 6 + 2 * kPw + 2 * kPw;   // doubles per sample

__host__ __device__ inline size_t prologue_scratch_bytes(int ts, int nd, int nl)
{
    // s_th[7][ts], s_Y[ts][nl], s_F[ts][nd] (complex), s_qp[ts][nd*nl],
    // the per-sample tables [ts][kProTab]
    return sizeof(double) * (size_t)ts * (7 + 2 * nl + 2 * nd + nd * nl + kProTab);
}

__device__ inline bool sample_ok(const ile_geom &g, const double th[7])
{
    bool fin = true;
#pragma unroll
    for (int p = 0; p < 7; p++) fin = fin && isfinite(th[p]);
    return fin && th[5] > 0.0 && th[4] >= -1.0 && th[4] <= 1.0 &&
           fabs(th[6]) <= g.t_ref_max;
}

// ------------------------------------------------------------- injection
// Zero-noise injection with a white unit-variance noise spectrum, so the
// inner product of Eq. (2) is <a|b> = sum_i conj(a_i) b_i (circular).
// Detector response to theta (Eqs. (5), (6) and the response below Eq. (6)):
//   d_k[i] = Re(F_k (D_ref/D) sum_a Y_a h_a[(i - lag_k) mod n]),
//   lag_k  = floor((t_ref + tau_k - t0)/dt + 1/2)  (the window rounding).
__global__ __launch_bounds__(256) void k_inject_resp(ile_geom g, const double2 *__restrict__ h,
                                                     int n, const double *__restrict__ th,
                                                     double *d)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)g.n_det * n) return;
    const int k = (int)(t / n), i = (int)(t % n);
    double fp, fx;
    antenna_dev(g, k, th[0], th[1], th[2], fp, fx);
    const double tau = delay_dev(g, k, th[0], th[1]);
    double x;
    {
#pragma clang fp contract(off)
        x = (th[6] + tau - g.t0) / g.dt;
    }
    const int64_t lag = (int64_t)floor(x + 0.5);
    int64_t src = ((int64_t)i - lag) % n;
    if (src < 0) src += n;
    const double kappa = g.d_ref / th[5];
    double re = 0.0, im = 0.0;
    for (int a = 0; a < g.n_lm; a++) {
        const double2 y = sylm_dev(g, a, th[4], th[3]);
        const double2 v = h[(size_t)a * n + src];
        re += y.x * v.x - y.y * v.y;
        im += y.x * v.y + y.y * v.x;
    }
    // Re(F z) with F = F+ + i Fx
    d[t] = kappa * (fp * re - fx * im);
}

// Q_k,a[s] = scale * sum_i conj(h_a[(i - s) mod n]) d_k[i]  (Eq. (8)): one
// workgroup per (k, a) and 256 consecutive s; d and the needed 511 h values
// of each 256-wide chunk of i are staged in LDS; sums run in i order.
__global__ __launch_bounds__(256) void k_inject_corr(int n_lm, int n, const double2 *__restrict__ h,
                                                     const double *__restrict__ d, double scale,
                                                     double2 *Q)
{
    __shared__ double sd[256];
    __shared__ double2 sh[512];
    const int ka = blockIdx.y, k = ka / n_lm, a = ka % n_lm;
    const int s0 = blockIdx.x * 256, t = threadIdx.x, s = s0 + t;
    double re = 0.0, im = 0.0;
    for (int i0 = 0; i0 < n; i0 += 256) {
        sd[t] = i0 + t < n ? d[(size_t)k * n + i0 + t] : 0.0;
        for (int j = t; j < 511; j += 256) {
            int64_t idx = ((int64_t)i0 - s0 - 255 + j) % n;
            if (idx < 0) idx += n;
            sh[j] = h[(size_t)a * n + idx];
        }
        __syncthreads();
        for (int ii = 0; ii < 256; ii++) {
            const double2 v = sh[ii - t + 255];
            re += v.x * sd[ii];
            im -= v.y * sd[ii];
        }
        __syncthreads();
    }
    if (s < n) Q[(size_t)ka * n + s] = make_double2(scale * re, scale * im);
}

// U_ab = sum_i conj(h_a[i]) h_b[i], V_ab = sum_i h_a[i] h_b[i] (Eq. (8));
// one workgroup per (a, b), fixed-order tree sum.
__global__ __launch_bounds__(256) void k_inject_gram(int n_lm, int n, const double2 *__restrict__ h,
                                                     double2 *U, double2 *V)
{
    __shared__ double red[4][256];
    const int a = blockIdx.x / n_lm, b = blockIdx.x % n_lm, t = threadIdx.x;
    double ur = 0, ui = 0, vr = 0, vi = 0;
    for (int i = t; i < n; i += 256) {
        const double2 x = h[(size_t)a * n + i], y = h[(size_t)b * n + i];
        ur += x.x * y.x + x.y * y.y;
        ui += x.x * y.y - x.y * y.x;
        vr += x.x * y.x - x.y * y.y;
        vi += x.x * y.y + x.y * y.x;
    }
    red[0][t] = ur;
    red[1][t] = ui;
    red[2][t] = vr;
    red[3][t] = vi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 4; q++) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0) {
        U[blockIdx.x] = make_double2(red[0][0], red[1][0]);
        V[blockIdx.x] = make_double2(red[2][0], red[3][0]);
    }
}

// ------------------------------------------------------------------ prep
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_prep(ile_geom g,
                                              const double *__restrict__ smp,
                                              int64_t N, int32_t *shifts,
                                              uint32_t *keys, uint32_t *hist,
                                              uint32_t n_buckets, int32_t *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double th[7];
#pragma unroll
    for (int p = 0; p < 7; p++) th[p] = smp[p * N + i];
    bool ok = sample_ok(g, th);
    int s[ILE_MAX_DET];
    for (int k = 0; k < g.n_det; k++) {
        s[k] = 0;
        if (ok) {
            double tau = delay_dev(g, k, th[0], th[1]);
            double x;
            {
#pragma clang fp contract(off)
                x = (th[6] + tau - g.t0) / g.dt;
            }
            double xs = floor(x + 0.5) - (double)g.half;
            if (xs >= 0.0 && xs <= (double)g.s_max)
                s[k] = (int)xs;
            else
                ok = false;
        }
    }
    uint32_t key = n_buckets - 1;   // invalid samples sort last
    if (ok) {
        key = cell_key(g, s);
    } else {
        atomicOr(err, 1);
    }
    for (int k = 0; k < g.n_det; k++) shifts[(int64_t)k * N + i] = ok ? s[k] : -1;
    keys[i] = key;
    (void)wave_count_slot(hist, key);
}

// Exclusive scan of n uint32 in place: blocks of 1024 threads x 4 values.
constexpr int kScanT = 1024;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanT * kScanPer;

__device__ inline uint32_t block_exscan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // Hillis-Steele over 1024 values in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanT; off <<= 1) {
        uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    total = sh[kScanT - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanT) void k_scan_local(uint32_t *v, int64_t n,
                                                       uint32_t *bsum)
{
    __shared__ uint32_t sh[kScanT];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    uint32_t x[kScanPer], run = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        x[j] = base + j < n ? v[base + j] : 0u;
        run += x[j];
    }
    uint32_t total;
    uint32_t ex = block_exscan(run, sh, total);
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        if (base + j < n) v[base + j] = ex;
        ex += x[j];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanT) void k_scan_top(uint32_t *bsum, int nb)
{
    // nb <= kScanBlock: one block, 4 values per thread
    __shared__ uint32_t sh[kScanT];
    int base = threadIdx.x * kScanPer;
    uint32_t x[kScanPer], run = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        x[j] = base + j < nb ? bsum[base + j] : 0u;
        run += x[j];
    }
    uint32_t total;
    uint32_t ex = block_exscan(run, sh, total);
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        if (base + j < nb) bsum[base + j] = ex;
        ex += x[j];
    }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *v, int64_t n,
                                                  const uint32_t *bsum)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] += bsum[i / kScanBlock];
}

__global__ __launch_bounds__(256) void k_scatter(const uint32_t *__restrict__ keys,
                                                 int64_t N, uint32_t *offs,
                                                 int32_t *perm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t pos = wave_count_slot(offs, keys[i]);
    perm[pos] = (int32_t)i;
}

// The scatter that also moves each sample's parameters and window starts
// to its place in tile order (read in sample order, so the terms pass then
// reads them coalesced instead of gathering them through perm).
__global__ __launch_bounds__(256) void k_scatter_copy(const uint32_t *__restrict__ keys,
                                                      int64_t N, uint32_t *offs, int32_t *perm,
                                                      const double *__restrict__ smp,
                                                      const int32_t *__restrict__ shifts, int nd,
                                                      double *__restrict__ smp_s,
                                                      int32_t *__restrict__ sh_s)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t pos = wave_count_slot(offs, keys[i]);
    perm[pos] = (int32_t)i;
#pragma unroll
    for (int p = 0; p < 7; p++) smp_s[(int64_t)p * N + pos] = smp[(int64_t)p * N + i];
    for (int k = 0; k < nd; k++) sh_s[(int64_t)k * N + pos] = shifts[(int64_t)k * N + i];
}

__global__ __launch_bounds__(256) void k_identity(int32_t *perm, int64_t N)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) perm[i] = (int32_t)i;
}

// ------------------------------------------------------------ contraction
// One workgroup = one tile of TS samples (in sorted order), NT threads.
// Q is stored planar per detector: row 2a holds Re Q_a, row 2a+1 Im Q_a,
// so Re(conj(c_a) Q_a[p]) = sum over the two rows of C[row] * Qm[row][p].
//
// G phase per (chunk, detector), two engines:
//   ENG_VALU: each thread owns one position p and accumulates G for all TS
//             samples with FMAs; coefficients broadcast from LDS.
//   ENG_MFMA: the G block is the real GEMM  C[TS x 2n_lm] * Qm[2n_lm x p]
//             on v_mfma_f64_16x16x4 (TS = 16 = M); each wave owns N-tiles of
//             16 positions, A (coefficients) from LDS, B (Q) from memory.
// Realign: thread j of the chunk adds G[alpha][s_alpha,k - s_min,k + j] for
// every sample; online FP64 log-sum-exp over the bins each thread owns.
// ENG_PH: the phased matrix-core engine below (FP64 or FP32 operands).
enum { ENG_VALU = 0, ENG_MFMA = 1, ENG_BF16 = 2, ENG_PH = 3 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// One 16x16x4 matrix-core step in the precision of the operands.  Output
// layouts on gfx950 (checked with lane-layout probes): f64 gives
// D[l/16 + 4v][l%16], f32 (and bf16 below) D[4(l/16) + v][l%16].
template <typename TQ> struct mfma_acc;
template <> struct mfma_acc<double> {
    using type = v4d;
    static __device__ inline v4d step(double a, double b, v4d c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int r, int v) { return r + 4 * v; }
};
template <> struct mfma_acc<float> {
    using type = v4f;
    static __device__ inline v4f step(float a, float b, v4f c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int r, int v) { return 4 * r + v; }
};

// G block on the matrix cores: Gs[alpha][p] = sum_r A[alpha][r] Qm[r][P0 + p]
// for p < W (<= NT), 16 samples.  v_mfma_f64_16x16x4 on gfx950 (checked
// with a lane-layout probe): lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[l/16 + 4v][l%16], v = 0..3.  Wave wv computes the N-tiles
// wv, wv+NW, ... (NU of them, wave-uniform) of 16 positions.  Q rows are
// padded with zeros to 4 KSP in memory, so every lane loads a valid row;
// columns past the end of Q are clamped (their results are never read).
template <typename TQ, int NT, int NU>
__device__ inline void mfma_tiles(TQ *Gs, const TQ *coefA, const TQ *Qk, int nq,
                                  int KSP, int P0, int lane, int wv)
{
    constexpr int NW = NT / 64;
    const int row = lane >> 4, col = lane & 15;
    using M = mfma_acc<TQ>;
    typename M::type acc[NU];
    const TQ *qb[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        acc[u] = typename M::type{0, 0, 0, 0};
        qb[u] = Qk + (int64_t)row * nq + min(P0 + 16 * (wv + NW * u) + col, nq - 1);
    }
    const int64_t step = 4 * (int64_t)nq;
    // three operand buffers, each reloaded right after its MFMAs consumed
    // it, so every load is in flight for two k-steps; the k-steps past KSP
    // of the last round are skipped by wave-uniform tests (prefetch indices
    // past the end are clamped and unused)
    const int kl = KSP - 1;
    TQ a0 = coefA[lane], a1 = coefA[min(1, kl) * 64 + lane], a2, b0[NU], b1[NU], b2[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        b0[u] = qb[u][0];
        b1[u] = qb[u][min(1, kl) * step];
    }
    // sched_barrier(0) keeps the compiler from folding the prefetch back
    // next to its use
    for (int ks = 0; ks < KSP; ks += 3) {
        const int k2 = min(ks + 2, kl), k3 = min(ks + 3, kl), k4 = min(ks + 4, kl);
        a2 = coefA[k2 * 64 + lane];
#pragma unroll
        for (int u = 0; u < NU; u++) b2[u] = qb[u][k2 * step];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NU; u++)
            acc[u] = M::step(a0, b0[u], acc[u]);
        __builtin_amdgcn_sched_barrier(0);
        a0 = coefA[k3 * 64 + lane];
#pragma unroll
        for (int u = 0; u < NU; u++) b0[u] = qb[u][k3 * step];
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < KSP) {
#pragma unroll
            for (int u = 0; u < NU; u++)
                acc[u] = M::step(a1, b1[u], acc[u]);
        }
        __builtin_amdgcn_sched_barrier(0);
        a1 = coefA[k4 * 64 + lane];
#pragma unroll
        for (int u = 0; u < NU; u++) b1[u] = qb[u][k4 * step];
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 2 < KSP) {
#pragma unroll
            for (int u = 0; u < NU; u++)
                acc[u] = M::step(a2, b2[u], acc[u]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int t = wv + NW * u;
#pragma unroll
        for (int v = 0; v < 4; v++) Gs[M::row(row, v) * NT + 16 * t + col] = (TQ)acc[u][v];
    }
}

template <typename TQ, int NT>
__device__ inline void mfma_gphase(TQ *Gs, const TQ *coefA, const TQ *Qk, int nq,
                                   int KSP, int P0, int W, int lane)
{
    constexpr int NW = NT / 64, TPW = NT / 16 / NW;
    static_assert(TPW == 4, "four N-tiles per wave");
    // wave index in an SGPR so the tile count below is known to be uniform
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntile = (W + 15) >> 4;
    int nu = ntile > wv ? (ntile - wv + NW - 1) / NW : 0;
    nu = __builtin_amdgcn_readfirstlane(nu < TPW ? nu : TPW);
    switch (nu) {
    case 4: mfma_tiles<TQ, NT, 4>(Gs, coefA, Qk, nq, KSP, P0, lane, wv); break;
    case 3: mfma_tiles<TQ, NT, 3>(Gs, coefA, Qk, nq, KSP, P0, lane, wv); break;
    case 2: mfma_tiles<TQ, NT, 2>(Gs, coefA, Qk, nq, KSP, P0, lane, wv); break;
    case 1: mfma_tiles<TQ, NT, 1>(Gs, coefA, Qk, nq, KSP, P0, lane, wv); break;
    default: break;
    }
}

// BF16 hi/lo contraction on v_mfma_f32_16x16x32_bf16: the K dimension is
// the concatenation [Q_hi; Q_lo; Q_hi] against [C_hi, C_hi, C_lo] (3 x 2 n_lm
// rows, zero-padded to 32 KSB), i.e. C.Q to about 16 significant bits with
// float accumulation.  Q is stored K-contiguous per position
// (Qb[p][32 KSB] bf16), so a lane's 8 consecutive k values are one 16-byte
// load; A comes from LDS in the same [ks][lane][8] order.
template <int NT, int NU>
__device__ inline void bf16_tiles(float *Gs, const v8bf *coefA, const v8bf *Qk, int nq, int KSB,
                                  int P0, int lane, int wv)
{
    constexpr int NW = NT / 64;
    const int row = lane >> 4, col = lane & 15;
    v4f acc[NU];
    const v8bf *qb[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        acc[u] = v4f{0, 0, 0, 0};
        qb[u] = Qk + (int64_t)min(P0 + 16 * (wv + NW * u) + col, nq - 1) * (4 * KSB) + row;
    }
    for (int ks = 0; ks < KSB; ks++) {
        const v8bf a = coefA[ks * 64 + lane];
        v8bf b[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) b[u] = qb[u][4 * ks];
#pragma unroll
        for (int u = 0; u < NU; u++) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[u], acc[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int t = wv + NW * u;
#pragma unroll
        for (int v = 0; v < 4; v++) Gs[(4 * row + v) * NT + 16 * t + col] = acc[u][v];
    }
}

template <int NT>
__device__ inline void bf16_gphase(float *Gs, const v8bf *coefA, const v8bf *Qk, int nq, int KSB,
                                   int P0, int W, int lane)
{
    constexpr int NW = NT / 64, TPW = NT / 16 / NW;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntile = (W + 15) >> 4;
    int nu = ntile > wv ? (ntile - wv + NW - 1) / NW : 0;
    nu = __builtin_amdgcn_readfirstlane(nu < TPW ? nu : TPW);
    switch (nu) {
    case 4: bf16_tiles<NT, 4>(Gs, coefA, Qk, nq, KSB, P0, lane, wv); break;
    case 3: bf16_tiles<NT, 3>(Gs, coefA, Qk, nq, KSB, P0, lane, wv); break;
    case 2: bf16_tiles<NT, 2>(Gs, coefA, Qk, nq, KSB, P0, lane, wv); break;
    case 1: bf16_tiles<NT, 1>(Gs, coefA, Qk, nq, KSB, P0, lane, wv); break;
    default: break;
    }
}

template <int ENG> __host__ __device__ inline size_t coef_bytes(int ts, int nd, int nl, size_t e)
{
    // VALU: complex [nd][nl][ts]; MFMA: real [nd][KSP][64]; BF16: [nd][KSB][64][8] bf16
    return ENG == ENG_VALU   ? (size_t)nd * nl * ts * 2 * e
           : ENG == ENG_MFMA ? (size_t)nd * ksp_of(nl) * 64 * e
                             : (size_t)nd * ksb_of(nl) * 64 * 8 * 2;
}

// Online log-sum-exp of one bin's contraction per sample (q is constant
// over bins and is subtracted at the end); one exp per sample and bin.
template <typename TQ, int TS>
__device__ __forceinline__ void lse_update(const TQ *L, double *m, double *sacc)
{
#pragma unroll
    for (int al = 0; al < TS; al++) {
        const double x = (double)L[al];
        const double d = x - m[al];
        const double e = exp(-fabs(d));
        const bool gt = d > 0.0;
        sacc[al] = gt ? fma(sacc[al], e, 1.0) : sacc[al] + e;
        m[al] = gt ? x : m[al];
    }
}

// Iterator over the pipeline items (chunk j0 of Jc bins, detector k,
// position block blk).
struct PipeIt {
    int j0, Jc, k, blk;
    bool valid;
};

__device__ __forceinline__ void pipe_first(PipeIt &it, int J, int n_t)
{
    it.j0 = 0;
    it.Jc = min(J, n_t);
    it.k = 0;
    it.blk = 0;
    it.valid = n_t > 0;
}

__device__ __forceinline__ void pipe_next(PipeIt &it, int J, int n_t, int nd,
                                          const int *spread, int NP)
{
    it.blk += NP;
    if (it.blk < it.Jc + spread[it.k]) return;
    it.blk = 0;
    if (++it.k < nd) return;
    it.k = 0;
    it.j0 += J;
    if (it.j0 < n_t) {
        it.Jc = min(J, n_t - it.j0);
        return;
    }
    it.valid = false;
}

__device__ __forceinline__ bool pipe_last_of_chunk(const PipeIt &it, int nd, int spread_last,
                                                   int NP)
{
    return it.k == nd - 1 && it.blk + NP >= it.Jc + spread_last;
}

// Deterministic reduction of the per-thread log-sum-exp states over the
// workgroup, in two halves separated by barriers: each wave writes its
// per-sample maximum (then its per-sample sum of s e^{m - M}) to s_red[wave]
// by a fixed butterfly; the M (then the result) are formed over the waves
// in wave order.  Threads with no state contribute -inf (then 0).
template <int TS>
__device__ inline void lse_wave_max(const double *m, double (*s_red)[TS], int lane, int wv)
{
#pragma unroll
    for (int al = 0; al < TS; al++) {
        double v = m ? m[al] : -INFINITY;
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        if (lane == 0) s_red[wv][al] = v;
    }
}
template <int TS>
__device__ inline void lse_wave_sum(const double *m, const double *sacc, const double *s_M,
                                    double (*s_red)[TS], int lane, int wv)
{
#pragma unroll
    for (int al = 0; al < TS; al++) {
        double v = 0.0;
        if (m) v = (m[al] == -INFINITY) ? 0.0 : sacc[al] * exp(m[al] - s_M[al]);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) s_red[wv][al] = v;
    }
}

// 16-lane reductions of doubles by DPP row rotations (8, 4, 2, 1 lanes) of
// both 32-bit halves: lane i meets the partner value of an xor butterfly
// (after the rotation by n the partials repeat with period n), so every lane
// of the row ends with the same bits.
template <int N>
__device__ inline double row_ror64(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x120 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x120 + N, 0xF, 0xF,
                                               false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline double row_max64(double x)
{
    x = fmax(x, row_ror64<8>(x));
    x = fmax(x, row_ror64<4>(x));
    x = fmax(x, row_ror64<2>(x));
    return fmax(x, row_ror64<1>(x));
}
__device__ inline double row_sum64(double x)
{
    x += row_ror64<8>(x);
    x += row_ror64<4>(x);
    x += row_ror64<2>(x);
    return x + row_ror64<1>(x);
}

// Matrix-core epilogue: the consumers' per-sample states go through LDS R
// (the free G buffers, [TS][NP] doubles); 16 lanes per sample (threads
// tid < 16 TS) combine the NP entries of their sample in a fixed order, then
// across the 16 lanes.  Pass 1 gives M = max m, pass 2 S = sum s e^{m - M}.
template <int TS, int NP>
__device__ inline double epi_reduce(const double *R, int tid, bool is_max)
{
    const int al = tid >> 4, l16 = tid & 15;
    double v = is_max ? -INFINITY : 0.0;
    for (int c = l16; c < NP; c += 16) {
        const double x = R[al * NP + c];
        v = is_max ? fmax(v, x) : v + x;
    }
    return is_max ? row_max64(v) : row_sum64(v);
}

// Per-sample part of a tile, shared by the engines: the samples, -2Y_lm,
// the antenna patterns, the coefficients c = (d_ref/D) F_k Y_lm in the
// engine's operand layout and the quadratic term q of Eq. (7).  scr is free
// LDS of scr_cap bytes (at least prologue_scratch_bytes); U_k and V_k are
// staged there too when they fit.  s_d receives the absolute window starts
// (0 for invalid samples).  Ends with a barrier.
template <typename TQ, int TS, int NT, int ENG>
__device__ __forceinline__ void tile_prologue(
    const ile_geom &g, int64_t base, const double *__restrict__ smp, int64_t N,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ shifts,
    const double2 *__restrict__ U, const double2 *__restrict__ V, double *scr,
    size_t scr_cap, TQ *coef, double *s_q, int *s_idx, int *s_ok, int (*s_d)[TS])
{
    const int tid = threadIdx.x;
    const int nd = g.n_det, nl = g.n_lm;
    const int KSP = ksp_of(nl);    // k-steps per detector (padded)
    const int KSB = ksb_of(nl);    // BF16 k-steps
    const size_t scr_bytes = prologue_scratch_bytes(TS, nd, nl);
    double *s_th = scr;                                  // [7][TS]
    double2 *s_Y = reinterpret_cast<double2 *>(scr + 7 * TS);   // [TS][nl]
    double2 *s_F = s_Y + TS * nl;                        // [TS][nd]
    double *s_qp = reinterpret_cast<double *>(s_F + TS * nd);   // [TS][nd*nl]
    double *s_tab = s_qp + TS * nd * nl;                 // [TS][kProTab]

    // 1. samples of the tile and, one thread per sample, the trigonometry
    //    every mode and detector of the sample shares
    if (tid < TS) {
        int64_t i = base + tid;
        int idx = -1, ok = 0;
        double th[7] = {0, 0, 0, 0, 0, 1, 0};
        if (i < N) {
            idx = perm[i];
#pragma unroll
            for (int p = 0; p < 7; p++) th[p] = smp[(int64_t)p * N + idx];
            ok = sample_ok(g, th);
            for (int k = 0; k < nd; k++) {
                int s = shifts[(int64_t)k * N + idx];
                ok = ok && s >= 0 && s <= g.s_max;
                s_d[k][tid] = s;
            }
        }
        s_idx[tid] = idx;
        s_ok[tid] = ok;
        if (!ok) {
            th[0] = th[1] = th[2] = th[3] = th[4] = th[6] = 0.0;
            th[5] = 1.0;
            for (int k = 0; k < nd; k++) s_d[k][tid] = 0;
        }
#pragma unroll
        for (int p = 0; p < 7; p++) s_th[p * TS + tid] = th[p];
        double *tb = s_tab + tid * kProTab;
        sincos(th[0] - g.gmst, &tb[0], &tb[1]);
        sincos(th[1], &tb[2], &tb[3]);
        sincos(th[2], &tb[4], &tb[5]);
        // powers of cos(iota/2), sin(iota/2) by repeated products from 1
        const double c = sqrt(0.5 * (1.0 + th[4])), sn = sqrt(0.5 * (1.0 - th[4]));
        double *cp = tb + 6, *sp = cp + kPw;
        double pc = 1.0, ps = 1.0;
        cp[0] = sp[0] = 1.0;
        for (int q = 1; q < kPw; q++) {
            pc *= c;
            ps *= sn;
            cp[q] = pc;
            sp[q] = ps;
        }
        // e^{i m phi} = (e^{i phi})^m, m = -ILE_LMAX .. ILE_LMAX
        double2 *em = reinterpret_cast<double2 *>(sp + kPw);
        double s1, c1;
        sincos(th[3], &s1, &c1);
        double er = 1.0, ei = 0.0;
        em[ILE_LMAX] = make_double2(1.0, 0.0);
        for (int m = 1; m <= ILE_LMAX; m++) {
            const double r2 = er * c1 - ei * s1, i2 = er * s1 + ei * c1;
            er = r2;
            ei = i2;
            em[ILE_LMAX + m] = make_double2(er, ei);
            em[ILE_LMAX - m] = make_double2(er, -ei);
        }
    }
    __syncthreads();

    // 2. harmonics -2Y_lm(iota, phi) (the Wigner-d sum over the mode's
    //    terms, then e^{i m phi}), or the surrogate form's basis vectors, and
    //    the antenna patterns F = F+ + i Fx
    for (int t = tid; t < TS * (nl + nd); t += NT) {
        if (t < TS * nl) {
            const int al = t / nl, a = t - al * nl;
            if (g.ext_y) {
                s_Y[al * nl + a] = s_ok[al] ? g.ext_y[(int64_t)s_idx[al] * nl + a]
                                            : make_double2(0.0, 0.0);
            } else {
                const double *cp = s_tab + al * kProTab + 6, *sp = cp + kPw;
                const int t0 = g.mode_first[a], nt = g.mode_nterm[a];
                double sum = 0.0;
                for (int u = t0; u < t0 + nt; u++)
                    sum += g.term_a[u] * cp[g.term_pw[u] & 255] * sp[g.term_pw[u] >> 8];
                const double2 e = reinterpret_cast<const double2 *>(sp + kPw)[ILE_LMAX + g.mode_m[a]];
                s_Y[al * nl + a] = make_double2(sum * e.x, sum * e.y);
            }
        } else {
            const int u = t - TS * nl;
            const int al = u / nd, k = u - al * nd;
            double fp, fx;
            antenna_trig(g, k, s_tab + al * kProTab, fp, fx);
            s_F[al * nd + k] = make_double2(fp, fx);
        }
    }
    __syncthreads();

    // 3. per detector: the coefficients c = (d_ref/D) F_k Y_lm in the
    //    engine's operand layout (modes a in [nl, 2 KSP) are the zero padding
    //    of the matrix-core K dimension), and the rows of the quadratic term
    //    of Eq. (7).  Only the Hermitian part of U and the symmetric part of V
    //    enter it (Re(Y^H U Y) = Y^H U_h Y, Y^T V Y = Y^T V_s Y), so each row
    //    a sums over b >= a only, the off-diagonal terms twice:
    //      row_a = |F|^2 (U_h,aa |Y_a|^2 + 2 Re(conj(Y_a) sum_{b>a} U_h,ab Y_b))
    //            + Re(F^2 (V_s,aa Y_a^2 + 2 Y_a sum_{b>a} V_s,ab Y_b)).
    //    A thread takes rows a and nl - 1 - a (nl - 1 terms together).
    if (ENG == ENG_BF16) {
        unsigned short *cz = reinterpret_cast<unsigned short *>(coef);
        for (int t = tid; t < nd * KSB * 64 * 8; t += NT) cz[t] = 0;
        __syncthreads();
    }
    const int nlp = ENG == ENG_MFMA ? 2 * KSP : nl;
    const int npr = (nl + 1) / 2;
    const size_t uv_off = (scr_bytes + 15) & ~(size_t)15;
    const bool stage_uv = uv_off + 2 * (size_t)nl * nl * sizeof(double2) <= scr_cap;
    double2 *s_U = reinterpret_cast<double2 *>(reinterpret_cast<unsigned char *>(scr) + uv_off);
    double2 *s_V = s_U + nl * nl;
    for (int k = 0; k < nd; k++) {
        const double2 *Uk = U + (int64_t)k * nl * nl, *Vk = V + (int64_t)k * nl * nl;
        if (stage_uv) {
            for (int e = tid; e < nl * nl; e += NT) {
                const int a = e / nl, b = e - a * nl;
                const double2 u1 = Uk[e], u2 = Uk[b * nl + a], v1 = Vk[e], v2 = Vk[b * nl + a];
                s_U[e] = make_double2(0.5 * (u1.x + u2.x), 0.5 * (u1.y - u2.y));
                s_V[e] = make_double2(0.5 * (v1.x + v2.x), 0.5 * (v1.y + v2.y));
            }
            __syncthreads();
        }
        // coefficients: samples fastest, so the 16 lanes of one (k, a)
        // write neighbouring operand slots
        for (int t = tid; t < TS * nlp; t += NT) {
            const int al = t % TS, a = t / TS;
            double cx = 0.0, cy = 0.0;
            if (a < nl) {
                const double kap = s_ok[al] ? g.d_ref / s_th[5 * TS + al] : 0.0;
                const double2 F = s_F[al * nd + k], Ya = s_Y[al * nl + a];
                cx = kap * (F.x * Ya.x - F.y * Ya.y);
                cy = kap * (F.x * Ya.y + F.y * Ya.x);
            }
            if (ENG == ENG_VALU) {
                coef[((k * nl + a) * TS + al) * 2] = (TQ)cx;
                coef[((k * nl + a) * TS + al) * 2 + 1] = (TQ)cy;
            } else if (ENG == ENG_BF16) {
                // A row k' of [C_hi, C_hi, C_lo]: lane = 16 (k' % 32 / 8) + alpha,
                // element k' % 8, k-step k' / 32
                __bf16 *cb = reinterpret_cast<__bf16 *>(coef) + (size_t)k * KSB * 64 * 8;
                const int R = 2 * nl;
                const double cv[2] = {cx, cy};
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const __bf16 hi = (__bf16)(float)cv[c];
                    const __bf16 lo = (__bf16)(float)(cv[c] - (double)(float)hi);
                    const int r = 2 * a + c;
                    const int kk[3] = {r, R + r, 2 * R + r};
                    const __bf16 vv[3] = {hi, hi, lo};
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        const int kp = kk[q];
                        cb[((kp >> 5) * 64 + ((kp & 31) >> 3) * 16 + al) * 8 + (kp & 7)] = vv[q];
                    }
                }
            } else {
                // A operand of k-step ks: lane = 16 * (row within the step) + alpha
                const int r0 = 2 * a;
                coef[(k * KSP + (r0 >> 2)) * 64 + (r0 & 3) * 16 + al] = (TQ)cx;
                coef[(k * KSP + (r0 >> 2)) * 64 + ((r0 & 3) + 1) * 16 + al] = (TQ)cy;
            }
        }
        // rows of the quadratic term, two per thread
        for (int t = tid; t < TS * npr; t += NT) {
            const int al = t % TS, pr = t / TS;
            const double2 F = s_F[al * nd + k];
            const double f2 = F.x * F.x + F.y * F.y;
            const double F2r = F.x * F.x - F.y * F.y, F2i = 2.0 * F.x * F.y;
            const double2 *Yr = s_Y + al * nl;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int a = h == 0 ? pr : nl - 1 - pr;
                if (h == 1 && a == pr) break;
                double ur = 0, ui = 0, vr = 0, vi = 0;
                for (int b = a + 1; b < nl; b++) {
                    const double2 Yb = Yr[b];
                    double2 u, v;
                    if (stage_uv) {
                        u = s_U[a * nl + b];
                        v = s_V[a * nl + b];
                    } else {
                        const double2 u1 = Uk[a * nl + b], u2 = Uk[b * nl + a];
                        const double2 v1 = Vk[a * nl + b], v2 = Vk[b * nl + a];
                        u = make_double2(0.5 * (u1.x + u2.x), 0.5 * (u1.y - u2.y));
                        v = make_double2(0.5 * (v1.x + v2.x), 0.5 * (v1.y + v2.y));
                    }
                    ur += u.x * Yb.x - u.y * Yb.y;
                    ui += u.x * Yb.y + u.y * Yb.x;
                    vr += v.x * Yb.x - v.y * Yb.y;
                    vi += v.x * Yb.y + v.y * Yb.x;
                }
                const double2 Ya = Yr[a];
                double2 ud, vd;
                if (stage_uv) {
                    ud = s_U[a * nl + a];
                    vd = s_V[a * nl + a];
                } else {
                    const double2 u1 = Uk[a * nl + a], v1 = Vk[a * nl + a];
                    ud = u1;
                    vd = v1;
                }
                // Y_a (V_s,aa Y_a + 2 w): the complex sum of the V part
                const double wr = vd.x * Ya.x - vd.y * Ya.y + 2.0 * vr;
                const double wi = vd.x * Ya.y + vd.y * Ya.x + 2.0 * vi;
                const double yvr = Ya.x * wr - Ya.y * wi, yvi = Ya.x * wi + Ya.y * wr;
                const double uq = ud.x * (Ya.x * Ya.x + Ya.y * Ya.y) + 2.0 * (Ya.x * ur + Ya.y * ui);
                s_qp[al * (nd * nl) + k * nl + a] = f2 * uq + (F2r * yvr - F2i * yvi);
            }
        }
        if (stage_uv) __syncthreads();   // before the next detector's copy
    }
    __syncthreads();

    static_assert(NT >= 16 * TS, "16 lanes per sample for the quadratic sum");
    if (tid < 16 * TS) {
        const int al = tid >> 4, l16 = tid & 15;
        double sum = 0.0;
        for (int r = l16; r < nd * nl; r += 16) sum += s_qp[al * (nd * nl) + r];
        for (int off = 8; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (l16 == 0) {
            const double kap = s_ok[al] ? g.d_ref / s_th[5 * TS + al] : 0.0;
            s_q[al] = 0.25 * kap * kap * sum;
        }
    }
    __syncthreads();
}

// ------------------------------------------------- per-sample terms
// The per-sample part of Eq. (7) for the phased engine, one lane per sample
// in tile order, so that it runs once per sample over the whole GPU rather
// than in one wave of each tile while the tile's other waves wait: the
// harmonics -2Y_lm(iota, phi) (Wigner-d terms times e^{i m phi}, or the
// surrogate form's vectors), the antenna patterns, the coefficient factors
// (d_ref/D) F_k and the quadratic term
//   q = (d_ref/D)^2 / 4 sum_k [ |F_k|^2 Y^H U_h,k Y + Re(F_k^2 Y^T V_s,k Y) ]
// with U_h the Hermitian part of U_k and V_s the symmetric part of V_k, so
// that only b >= a enters (the off-diagonal terms twice): per detector the
// host packs the upper triangles row by row, entry (a, b >= a) at
// 4 (a nl - a (a - 1) / 2 + b - a) as (Re U_h, Im U_h, Re V_s, Im V_s).
// Output: tile-major, field f of position t0 + r at
// terms[16 F (r / 16) + 16 f + r % 16].

// One lane's sample: its validity, window starts, the sines and cosines of
// the antenna angles, d_ref/D, and the tables the harmonics are read from:
// powers of cos and sin of iota/2 and e^{i m phi}, register arrays (of the
// caller, so that they stay in registers) read at indices that are the same
// in every lane.
struct TermsSample {
    int idx, ok;
    int sd[ILE_MAX_DET];
    double tr[6], kap;
};

__device__ __forceinline__ void terms_intake(const ile_geom &g, const double *__restrict__ smp,
                                             int64_t N, const int32_t *__restrict__ perm,
                                             const int32_t *__restrict__ shifts, int64_t i,
                                             bool in_order, TermsSample &S, double (&cp)[kPw],
                                             double (&sp)[kPw], double (&er)[kPw],
                                             double (&ei)[kPw])
{
    const int nd = g.n_det;
    S.idx = perm[i];
    // in_order: smp and shifts are already in tile order (a coalesced read);
    // else gathered through the permutation
    const int64_t src = in_order ? i : S.idx;
    double th[7];
#pragma unroll
    for (int p = 0; p < 7; p++) th[p] = smp[(int64_t)p * N + src];
#pragma unroll
    for (int k = 0; k < ILE_MAX_DET; k++) S.sd[k] = k < nd ? shifts[(int64_t)k * N + src] : 0;
    bool ok = sample_ok(g, th);
#pragma unroll
    for (int k = 0; k < ILE_MAX_DET; k++)
        ok = ok & (k >= nd || (S.sd[k] >= 0 && S.sd[k] <= g.s_max));
    S.ok = ok;
    if (!ok) {
        th[0] = th[1] = th[2] = th[3] = th[4] = th[6] = 0.0;
        th[5] = 1.0;
    }
    sincos(th[0] - g.gmst, &S.tr[0], &S.tr[1]);
    sincos(th[1], &S.tr[2], &S.tr[3]);
    sincos(th[2], &S.tr[4], &S.tr[5]);
    S.kap = ok ? g.d_ref / th[5] : 0.0;
    // powers of cos(iota/2), sin(iota/2) by repeated products from 1, and
    // e^{i m phi} = (e^{i phi})^m, |m| <= ILE_LMAX
    const double c = sqrt(0.5 * (1.0 + th[4])), sn = sqrt(0.5 * (1.0 - th[4]));
    cp[0] = sp[0] = 1.0;
#pragma unroll
    for (int q = 1; q < kPw; q++) {
        cp[q] = cp[q - 1] * c;
        sp[q] = sp[q - 1] * sn;
    }
    double s1, c1;
    sincos(th[3], &s1, &c1);
    er[ILE_LMAX] = 1.0;
    ei[ILE_LMAX] = 0.0;
#pragma unroll
    for (int m = 1; m <= ILE_LMAX; m++) {
        const double pr = er[ILE_LMAX + m - 1], pi = ei[ILE_LMAX + m - 1];
        er[ILE_LMAX + m] = pr * c1 - pi * s1;
        ei[ILE_LMAX + m] = pr * s1 + pi * c1;
        er[ILE_LMAX - m] = er[ILE_LMAX + m];
        ei[ILE_LMAX - m] = -ei[ILE_LMAX + m];
    }
}

// -2Y_lm of mode a: the mode's Wigner-d terms, then e^{i m phi}; or the
// surrogate form's vector entry.
__device__ __forceinline__ double2 terms_harmonic(const ile_geom &g, const TermsSample &S, int a,
                                                  const double (&cp)[kPw],
                                                  const double (&sp)[kPw],
                                                  const double (&er)[kPw],
                                                  const double (&ei)[kPw])
{
    if (g.ext_y) return S.ok ? g.ext_y[(int64_t)S.idx * g.n_lm + a] : make_double2(0.0, 0.0);
    const int u0 = g.mode_first[a], nt = g.mode_nterm[a];
    double sum = 0.0;
    for (int u = u0; u < u0 + nt; u++)
        sum += g.term_a[u] * cp[g.term_pw[u] & 255] * sp[g.term_pw[u] >> 8];
    const int mi = ILE_LMAX + g.mode_m[a];
    return make_double2(sum * er[mi], sum * ei[mi]);
}

// Row a of detector k's part of the quadratic term (the b > a sums w_U, w_V
// over the row's entries given), with f2 = |F|^2 and F^2 = (F2r, F2i).
__device__ __forceinline__ double terms_row(double2 Ya, double4 d, double ur, double ui,
                                            double vr, double vi, double f2, double F2r,
                                            double F2i)
{
    // Y_a (V_s,aa Y_a + 2 w_V): the complex sum of the V part
    const double wr = d.z * Ya.x - d.w * Ya.y + 2.0 * vr;
    const double wi = d.z * Ya.y + d.w * Ya.x + 2.0 * vi;
    const double yvr = Ya.x * wr - Ya.y * wi, yvi = Ya.x * wi + Ya.y * wr;
    const double uq = d.x * (Ya.x * Ya.x + Ya.y * Ya.y) + 2.0 * (Ya.x * ur + Ya.y * ui);
    return f2 * uq + (F2r * yvr - F2i * yvi);
}

__device__ __forceinline__ void terms_mac(double2 Yb, double4 e, double &ur, double &ui,
                                          double &vr, double &vi)
{
    ur = fma(e.x, Yb.x, fma(-e.y, Yb.y, ur));
    ui = fma(e.x, Yb.y, fma(e.y, Yb.x, ui));
    vr = fma(e.z, Yb.x, fma(-e.w, Yb.y, vr));
    vi = fma(e.z, Yb.y, fma(e.w, Yb.x, vi));
}

__device__ __forceinline__ void terms_store(const ile_geom &g, const TermsSample &S, double q,
                                            double *tp)
{
    const int nd = g.n_det, nl = g.n_lm;
    tp[0] = 0.25 * S.kap * S.kap * q;
    tp[16] = S.ok ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < ILE_MAX_DET; k++)
        if (k < nd) tp[(2 + 2 * nd + 2 * nl + k) * 16] = S.ok ? (double)S.sd[k] : 0.0;
}

__device__ __forceinline__ double *terms_slot(const ile_geom &g, double *terms, int64_t r)
{
    return terms + (r >> 4) * (16 * (int64_t)(2 + 3 * g.n_det + 2 * g.n_lm)) + (r & 15);
}

// Entry i of the triangles by vector loads at a uniform address (one cache
// line serves the wave): unlike scalar loads, which complete out of order,
// they can be waited for one step at a time.
__device__ __forceinline__ double4 tri_ld(__amdgpu_buffer_rsrc_t r, int i)
{
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 lo = __builtin_amdgcn_raw_buffer_load_b128(r, 0, i * 32, 0);
    const u4 hi = __builtin_amdgcn_raw_buffer_load_b128(r, 0, i * 32 + 16, 0);
    const double2 x = __builtin_bit_cast(double2, lo), y = __builtin_bit_cast(double2, hi);
    return make_double4(x.x, x.y, y.x, y.y);
}

constexpr int kTermsT = 64;    // lanes per block

// Any number of modes: a lane's harmonics are an LDS row of 64 lanes
// (conflict free, and no lane reads another's: no barrier); the triangles
// are read four entries per step, one step ahead (tri_ld).
__global__ __launch_bounds__(kTermsT) void k_terms(
    ile_geom g, const double *__restrict__ smp, int64_t N, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ shifts, bool in_order, const double4 *__restrict__ uvt,
    int64_t t0, int64_t n, double *__restrict__ terms)
{
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int lane = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * kTermsT + lane;   // position t0 + r
    if (r >= n) return;
    const int nd = g.n_det, nl = g.n_lm, ntri = nl * (nl + 1) / 2;
    double2 *Yl = reinterpret_cast<double2 *>(dyn_lds);   // [nl][64]
    const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double4 *>(uvt), (short)0, nd * ntri * (int)sizeof(double4), 0x00020000);
    double *tp = terms_slot(g, terms, r);
    TermsSample S;
    double cp[kPw], sp[kPw], er[kPw], ei[kPw];
    terms_intake(g, smp, N, perm, shifts, t0 + r, in_order, S, cp, sp, er, ei);
    for (int a = 0; a < nl; a++) {
        const double2 y = terms_harmonic(g, S, a, cp, sp, er, ei);
        Yl[a * kTermsT + lane] = y;
        tp[(2 + 2 * nd + 2 * a) * 16] = y.x;
        tp[(3 + 2 * nd + 2 * a) * 16] = y.y;
    }
    double qs = 0.0;
    for (int k = 0; k < nd; k++) {
        double fp, fx;
        antenna_trig(g, k, S.tr, fp, fx);
        tp[(2 + 2 * k) * 16] = S.kap * fp;
        tp[(3 + 2 * k) * 16] = S.kap * fx;
        const double f2 = fp * fp + fx * fx, F2r = fp * fp - fx * fx, F2i = 2.0 * fp * fx;
        int ro = k * ntri;   // row a's first entry (its diagonal)
        for (int a = 0; a < nl; a++) {
            double ur = 0, ui = 0, vr = 0, vi = 0;
            int b = a + 1;
            if (b + 3 < nl) {
                // four entries per step, the next step's loads issued before
                // this step's products (sums still in the order of b)
                double2 Yb[4];
                double4 e[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    Yb[q] = Yl[(b + q) * kTermsT + lane];
                    e[q] = tri_ld(rt, ro + b + q - a);
                }
                for (; b + 7 < nl; b += 4) {
                    double2 Yn[4];
                    double4 en[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        Yn[q] = Yl[(b + 4 + q) * kTermsT + lane];
                        en[q] = tri_ld(rt, ro + b + 4 + q - a);
                    }
#pragma unroll
                    for (int q = 0; q < 4; q++) terms_mac(Yb[q], e[q], ur, ui, vr, vi);
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        Yb[q] = Yn[q];
                        e[q] = en[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; q++) terms_mac(Yb[q], e[q], ur, ui, vr, vi);
                b += 4;
            }
            for (; b < nl; b++) terms_mac(Yl[b * kTermsT + lane], uvt[ro + b - a], ur, ui, vr, vi);
            qs += terms_row(Yl[a * kTermsT + lane], uvt[ro], ur, ui, vr, vi, f2, F2r, F2i);
            ro += nl - a;
        }
    }
    terms_store(g, S, qs, tp);
}

static size_t terms_lds_bytes(const ile_geom &g)
{
    return (size_t)kTermsT * g.n_lm * sizeof(double2);
}

// One tile: samples perm[base .. base + TS) of a point (those below N).
template <typename TQ, int TS, int NT, int ENG, bool DUMP>
__device__ __forceinline__ void contract_tile(
    const ile_geom &g, int64_t base, const double *__restrict__ smp, int64_t N,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ shifts,
    const TQ *__restrict__ Q, const double2 *__restrict__ U,
    const double2 *__restrict__ V, double *__restrict__ out,
    double *__restrict__ series)
{
    static_assert(ENG == ENG_VALU || (TS == 16 && NT % 128 == 0), "MFMA tile is 16 samples");
    static_assert(ENG != ENG_BF16 || sizeof(TQ) == 4, "BF16 engine accumulates in float");
    constexpr int NW = NT / 64;
    __shared__ __align__(16) TQ Gs[TS * NT];
    __shared__ double s_q[TS];
    __shared__ int s_idx[TS];      // sample index, -1 if the slot is empty
    __shared__ int s_ok[TS];
    __shared__ int s_d[ILE_MAX_DET][TS];
    __shared__ int s_smin[ILE_MAX_DET], s_spread[ILE_MAX_DET];
    __shared__ double s_red[NW][TS];
    __shared__ double s_M[TS];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    TQ *coef = reinterpret_cast<TQ *>(dyn_lds);

    const int tid = threadIdx.x;
    const int nd = g.n_det, nl = g.n_lm, nq = g.n_q;
    const int KSP = ksp_of(nl), RP = 4 * KSP;   // k-steps and Q rows per detector (padded)
    const int KSB = ksb_of(nl);                 // BF16 k-steps
    constexpr bool MF = ENG != ENG_VALU;        // matrix-core engines

    // prologue scratch: inside Gs when it fits, else after the coefficients
    const size_t scr_bytes = prologue_scratch_bytes(TS, nd, nl);
    double *scr = scr_bytes <= sizeof(Gs)
                      ? reinterpret_cast<double *>(Gs)
                      : reinterpret_cast<double *>(dyn_lds + coef_bytes<ENG>(TS, nd, nl, sizeof(TQ)));

    tile_prologue<TQ, TS, NT, ENG>(g, base, smp, N, perm, shifts, U, V, scr,
                                   scr == reinterpret_cast<double *>(Gs) ? sizeof(Gs) : 0,
                                   coef, s_q, s_idx, s_ok, s_d);

    // 4. per-detector window range of the tile
    if (tid < nd) {
        const int k = tid;
        int lo = 0x7fffffff, hi = -1;
        for (int al = 0; al < TS; al++)
            if (s_ok[al]) {
                lo = min(lo, s_d[k][al]);
                hi = max(hi, s_d[k][al]);
            }
        if (hi < 0) lo = hi = 0;
        s_smin[k] = lo;
        s_spread[k] = hi - lo;
    }
    __syncthreads();
    if (tid < TS)
        for (int k = 0; k < nd; k++) s_d[k][tid] = s_ok[tid] ? s_d[k][tid] - s_smin[k] : 0;
    __syncthreads();

    int smax_all = 0;
    for (int k = 0; k < nd; k++) smax_all = max(smax_all, s_spread[k]);
    // NP positions per G block: every thread for the vector engine, the
    // producer half of the workgroup for the matrix-core engine
    constexpr int NP = MF ? NT / 2 : NT;
    int J = NP - smax_all;
    if (J < 64) J = 64;

    const int lane = tid & 63, wv = tid >> 6;
    // the result of sample al: (M - q) + log S - log n_t, S = the block sum
    const auto finish_sample = [&](int al, double S) {
        if (s_idx[al] >= 0)
            out[s_idx[al]] = s_ok[al] ? (s_M[al] - s_q[al]) + log(S) - log((double)g.n_t) : NAN;
    };

    if constexpr (ENG == ENG_VALU) {
        double m[TS], sacc[TS];
#pragma unroll
        for (int al = 0; al < TS; al++) {
            m[al] = -INFINITY;
            sacc[al] = 0.0;
        }
        for (int j0 = 0; j0 < g.n_t; j0 += J) {
            const int Jc = min(J, g.n_t - j0);
            // thread tid owns the bins j == tid (mod NT); its bin in this chunk
            const int jrel = ((tid - j0) % NT + NT) % NT;
            const bool has = jrel < Jc;
            TQ L[TS];
#pragma unroll
            for (int al = 0; al < TS; al++) L[al] = (TQ)0;

            for (int k = 0; k < nd; k++) {
                const int Pk = s_smin[k] + j0;
                const int Wk = Jc + s_spread[k];
                const TQ *Qk = Q + (int64_t)k * RP * nq;
                for (int blk = 0; blk < Wk; blk += NT) {
                    const int p = blk + tid;
                    TQ acc[TS];
#pragma unroll
                    for (int al = 0; al < TS; al++) acc[al] = (TQ)0;
                    if (p < Wk) {
                        const TQ *qp = Qk + Pk + p;
                        const TQ *cf = coef + (size_t)k * nl * TS * 2;
                        TQ qnr = qp[0], qni = qp[nq];
                        for (int a = 0; a < nl; a++) {
                            const TQ qr = qnr, qi = qni;
                            // next mode's values are in flight during this mode's FMAs
                            if (a + 1 < nl) {
                                qnr = qp[(int64_t)(2 * a + 2) * nq];
                                qni = qp[(int64_t)(2 * a + 3) * nq];
                            }
                            const TQ *ca = cf + a * TS * 2;
#pragma unroll
                            for (int al = 0; al < TS; al++)
                                acc[al] = fma(ca[2 * al], qr, fma(ca[2 * al + 1], qi, acc[al]));
                        }
                    }
#pragma unroll
                    for (int al = 0; al < TS; al++) Gs[al * NT + tid] = acc[al];
                    __syncthreads();
                    if (has) {
#pragma unroll
                        for (int al = 0; al < TS; al++) {
                            const int ix = s_d[k][al] + jrel - blk;
                            const bool in = (unsigned)ix < (unsigned)NT;
                            const TQ v = Gs[al * NT + (in ? ix : 0)];
                            L[al] += in ? v : (TQ)0;
                        }
                    }
                    __syncthreads();
                }
            }
            if (has) {
                const int j = j0 + jrel;
                if (DUMP) {
                    for (int al = 0; al < TS; al++)
                        if (s_ok[al]) series[(int64_t)s_idx[al] * g.n_t + j] = (double)L[al] - s_q[al];
                }
                lse_update<TQ, TS>(L, m, sacc);
            }
        }
        lse_wave_max<TS>(m, s_red, lane, wv);
        __syncthreads();
        if (tid < TS) {
            double M = s_red[0][tid];
            for (int w = 1; w < NW; w++) M = fmax(M, s_red[w][tid]);
            s_M[tid] = M;
        }
        __syncthreads();
        lse_wave_sum<TS>(m, sacc, s_M, s_red, lane, wv);
        __syncthreads();
        if (tid < TS) {
            double S = s_red[0][tid];
            for (int w = 1; w < NW; w++) S += s_red[w][tid];
            finish_sample(tid, S);
        }
    } else {
        // Producer/consumer pipeline over the items (chunk, detector, block):
        // at step s the producer waves compute item s into Gs buffer s % 2
        // on the matrix cores while the consumer waves realign item s-1 from
        // the other buffer (and run the log-sum-exp at the end of a chunk);
        // one barrier per step.  Both iterators are advanced identically by
        // every thread, so the loop bounds are uniform.
        const bool producer = __builtin_amdgcn_readfirstlane(tid) < NP;
        static_assert(TS * NP * sizeof(double) <= sizeof(Gs), "epilogue states fit the G buffers");
        // Separate loops per role (wave-uniform branch) so that the consumer
        // state and the producer's operand buffers are never live together;
        // both loops take the same steps and meet at one barrier per step.
        PipeIt pi, ci;
        pipe_first(pi, J, g.n_t);
        pipe_first(ci, J, g.n_t);
        if (producer) {
            for (int step = 0; pi.valid || ci.valid; step++) {
                if (pi.valid) {
                    const int k = pi.k;
                    const int P0 = s_smin[k] + pi.j0 + pi.blk;
                    const int W = min(pi.Jc + s_spread[k] - pi.blk, NP);
                    if constexpr (ENG == ENG_BF16)
                        bf16_gphase<NP>(reinterpret_cast<float *>(Gs) + (step & 1) * (TS * NP),
                                        reinterpret_cast<const v8bf *>(coef) + (size_t)k * KSB * 64,
                                        reinterpret_cast<const v8bf *>(Q) + (int64_t)k * nq * 4 * KSB,
                                        nq, KSB, P0, W, lane);
                    else
                        mfma_gphase<TQ, NP>(Gs + (step & 1) * (TS * NP), coef + (size_t)k * KSP * 64,
                                            Q + (int64_t)k * RP * nq, nq, KSP, P0, W, lane);
                    pipe_next(pi, J, g.n_t, nd, s_spread, NP);
                }
                if (step > 0 && ci.valid) pipe_next(ci, J, g.n_t, nd, s_spread, NP);
                __syncthreads();
            }
            // epilogue (the consumers write R between the barriers); threads
            // tid < 16 TS reduce
            const double *R = reinterpret_cast<const double *>(Gs);
            __syncthreads();
            if (tid < 16 * TS) {
                const double M = epi_reduce<TS, NP>(R, tid, true);
                if ((tid & 15) == 0) s_M[tid >> 4] = M;
            }
            __syncthreads();
            __syncthreads();
            if (tid < 16 * TS) {
                const double S = epi_reduce<TS, NP>(R, tid, false);
                if ((tid & 15) == 0) finish_sample(tid >> 4, S);
            }
        } else {
            const int tc = tid - NP;   // consumer index
            double m[TS], sacc[TS];
#pragma unroll
            for (int al = 0; al < TS; al++) {
                m[al] = -INFINITY;
                sacc[al] = 0.0;
            }
            TQ L[TS];
#pragma unroll
            for (int al = 0; al < TS; al++) L[al] = (TQ)0;
            for (int step = 0; pi.valid || ci.valid; step++) {
                if (step > 0 && ci.valid) {
                    const TQ *G = Gs + ((step - 1) & 1) * (TS * NP);
                    const int jrel = ((tc - ci.j0) % NP + NP) % NP;
                    const bool has = jrel < ci.Jc;
                    if (has) {
#pragma unroll
                        for (int al = 0; al < TS; al++) {
                            const int ix = s_d[ci.k][al] + jrel - ci.blk;
                            const bool in = (unsigned)ix < (unsigned)NP;
                            const TQ v = G[al * NP + (in ? ix : 0)];
                            L[al] += in ? v : (TQ)0;
                        }
                    }
                    if (pipe_last_of_chunk(ci, nd, s_spread[nd - 1], NP)) {
                        if (has) {
                            const int j = ci.j0 + jrel;
                            if (DUMP) {
                                for (int al = 0; al < TS; al++)
                                    if (s_ok[al])
                                        series[(int64_t)s_idx[al] * g.n_t + j] =
                                            (double)L[al] - s_q[al];
                            }
                            lse_update<TQ, TS>(L, m, sacc);
                        }
#pragma unroll
                        for (int al = 0; al < TS; al++) L[al] = (TQ)0;
                    }
                    pipe_next(ci, J, g.n_t, nd, s_spread, NP);
                }
                if (pi.valid) pipe_next(pi, J, g.n_t, nd, s_spread, NP);
                __syncthreads();
            }
            // epilogue: the same three barriers as the producers
            double *R = reinterpret_cast<double *>(Gs);
#pragma unroll
            for (int al = 0; al < TS; al++) R[al * NP + tc] = m[al];
            __syncthreads();
            if (tid < 16 * TS) {
                const double M = epi_reduce<TS, NP>(R, tid, true);
                if ((tid & 15) == 0) s_M[tid >> 4] = M;
            }
            __syncthreads();
#pragma unroll
            for (int al = 0; al < TS; al++)
                R[al * NP + tc] = m[al] == -INFINITY ? 0.0 : sacc[al] * exp(m[al] - s_M[al]);
            __syncthreads();
            if (tid < 16 * TS) {
                const double S = epi_reduce<TS, NP>(R, tid, false);
                if ((tid & 15) == 0) finish_sample(tid >> 4, S);
            }
        }
    }
}

// ------------------------------------------------ phased matrix-core engine
// One workgroup of four waves per tile of 16 samples.  On gfx950 an FP64
// matrix-core step holds its SIMD's issue for its whole duration, so the
// vector work and the matrix work of a SIMD add up instead of overlapping.
// The tile is therefore not split into producer and consumer waves (which
// leaves the matrix work on some SIMDs and the vector work on others):
// every wave takes both roles in turn, per chunk of J bins:
//   G phase, one detector k at a time: the windowed products
//            G_k[alpha][p] = sum_r C_k[alpha][r] Qm_k[r][P_k + p] over the
//            union of the chunk's windows (P_k = smin_k + j0), as 16-wide
//            N-tiles dealt to the waves in turn, each result moved to its
//            sample's chunk bin: X[alpha][jj] with jj = p - (s_alpha,k -
//            smin_k), stored for the first detector and added for the
//            others (a barrier between detectors), so X holds the sum over
//            the detectors in ascending order;
//   L phase: lane (alpha, sub), LPS = 16 or 32 lanes per sample, owns the
//            bins j = sub (mod LPS) and folds X[alpha][j - j0] into its
//            log-sum-exp.
// X has one row of J bins per sample whatever the spread of the tile's
// window starts (which only widens the unions), so J is set by the LDS
// budget alone.
//
// Log-sum-exp with a lagging reference: each lane keeps (m, s) with
// s = sum exp(x - m) over its bins, and moves m to x only at its first bin
// or when x > m + kLseSlack, so most bins cost one exp and one add.  The
// 16 lanes of a sample are merged by a fixed tree at the end.  A sample's
// bins, their order within each lane and the merge depend neither on the
// tile it lands in nor on the chunking or the pass, and neither does its
// result.
constexpr double kLseSlack = 64.0;

// a * b + c with c a wave-uniform constant held in scalar registers.  The
// compiler's own selection turns Horner steps into a register copy of the
// constant plus an accumulating FMA (its tied operand); this form needs no
// copy.  Arithmetic only.
__device__ __forceinline__ double fma_sc(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// e^d for d <= kLseSlack, the log-sum-exp's terms: d = n ln2 + r with
// n = rint(d / ln2) and r reduced in two parts (Cody and Waite), so
// |r| <= ln2 / 2; e^r by its Taylor polynomial of degree 13 (truncation
// below 5e-18 relative); then scaled by 2^n.  Arguments below -1000 are
// clamped there (the result underflows to 0 either way), so no overflow or
// NaN test is needed.  Relative error a few ulp.
__device__ __forceinline__ double exp_lse(double d)
{
    // d is never NaN here, so the clamp needs no canonicalization
    asm("v_max_f64 %0, %1, %2" : "=v"(d) : "v"(d), "s"(-1000.0));
    const double n = rint(d * 1.4426950408889634074);
    const double r = fma(-n, 1.9082149292705877000e-10, fma(-n, 6.9314718036912381649e-1, d));
    double p = fma_sc(r, 1.0 / 6227020800.0, 1.0 / 479001600.0);   // 1/13!, 1/12!
    p = fma_sc(p, r, 1.0 / 39916800.0);
    p = fma_sc(p, r, 1.0 / 3628800.0);
    p = fma_sc(p, r, 1.0 / 362880.0);
    p = fma_sc(p, r, 1.0 / 40320.0);
    p = fma_sc(p, r, 1.0 / 5040.0);
    p = fma_sc(p, r, 1.0 / 720.0);
    p = fma_sc(p, r, 1.0 / 120.0);
    p = fma_sc(p, r, 1.0 / 24.0);
    p = fma_sc(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

template <typename TQ> struct qload;
template <> struct qload<double> {
    static __device__ inline double ld(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
        return __builtin_bit_cast(double, v);
    }
};
template <> struct qload<float> {
    static __device__ inline float ld(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
};

// Buffer resource over one detector's Q rows (raw bytes, gfx9 word 3).
template <typename TQ>
__device__ inline __amdgpu_buffer_rsrc_t q_rsrc(const TQ *Qk, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<TQ *>(Qk), (short)0, bytes, 0x00020000);
}

// NU N-tiles t[u] of detector k, computed together so that NU accumulations
// are in flight: lane l supplies A[l%16][l/16] (the detector's
// coefficients, LDS; one read per k-step serves all NU tiles) and
// B[l/16][l%16] = Qm_k[4 ks + l/16][P0 + 16 t + l%16] by buffer loads, the
// lane's offset in a VGPR and the k-step's in an SGPR, so a load costs no
// vector instruction.  Columns past the end of Q are clamped (past every
// sample's window: never moved to X).  Operands are double-buffered: the
// loads of k-step ks + 1 are issued before the products of k-step ks.  The
// result D[alpha][16 t + c] goes to X[alpha][16 t + c - dd[v]] (alpha =
// row(lane / 16, v), dd its window start minus smin_k) when that bin is in
// [0, Jc): stored when `add` is false, else added.  Each (alpha, bin) comes
// from exactly one lane of one tile.  BF: the stores without branches, into
// X's one element past its 16 rows of xrow bins when out of range.
template <typename TQ, int NU, bool BF>
__device__ inline void ph_tiles(TQ *X, int xrow, const TQ *coefk, __amdgpu_buffer_rsrc_t rs,
                                int qrow0, int nq, int KSP, int P0, const int (&t)[4],
                                const int (&dd)[4], int Jc, bool add, int lane)
{
    using M = mfma_acc<TQ>;
    const int row = lane >> 4, col = lane & 15;
    typename M::type acc[NU];
    int vo[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        acc[u] = typename M::type{0, 0, 0, 0};
        vo[u] = ((qrow0 + row) * nq + min(P0 + 16 * t[u] + col, nq - 1)) * (int)sizeof(TQ);
    }
    const int kstep = 4 * nq * (int)sizeof(TQ);
    TQ a0 = coefk[lane], a1, b0[NU], b1[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) b0[u] = qload<TQ>::ld(rs, vo[u], 0);
    // k-steps in pairs with every load and product unconditional (a load
    // under a branch is sunk next to its use); an odd last step follows
    int ks = 0;
    for (; ks + 1 < KSP; ks += 2) {
        const int k2 = min(ks + 2, KSP - 1);
        a1 = coefk[(ks + 1) * 64 + lane];
#pragma unroll
        for (int u = 0; u < NU; u++) b1[u] = qload<TQ>::ld(rs, vo[u], (ks + 1) * kstep);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NU; u++) acc[u] = M::step(a0, b0[u], acc[u]);
        __builtin_amdgcn_sched_barrier(0);
        a0 = coefk[k2 * 64 + lane];
#pragma unroll
        for (int u = 0; u < NU; u++) b0[u] = qload<TQ>::ld(rs, vo[u], k2 * kstep);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NU; u++) acc[u] = M::step(a1, b1[u], acc[u]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (ks < KSP) {
#pragma unroll
        for (int u = 0; u < NU; u++) acc[u] = M::step(a0, b0[u], acc[u]);
    }
    if constexpr (BF) {
        // without branches: a value whose bin is outside [0, Jc) goes to the
        // slot past the 16 rows (never read as a bin); when adding, every
        // load is issued before the first sum
        int a[NU][4];
#pragma unroll
        for (int u = 0; u < NU; u++) {
            const int c = 16 * t[u] + col;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int jj = c - dd[v];
                a[u][v] = (unsigned)jj < (unsigned)Jc ? M::row(row, v) * xrow + jj : 16 * xrow;
            }
        }
        if (add) {
            TQ o[NU][4];
#pragma unroll
            for (int u = 0; u < NU; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) o[u][v] = X[a[u][v]];
#pragma unroll
            for (int u = 0; u < NU; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) X[a[u][v]] = o[u][v] + (TQ)acc[u][v];
        } else {
#pragma unroll
            for (int u = 0; u < NU; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) X[a[u][v]] = (TQ)acc[u][v];
        }
    } else {
        // the branch form needs fewer registers (FP32 tiles run three
        // workgroups per CU; the series form holds more state)
#pragma unroll
        for (int u = 0; u < NU; u++) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int jj = 16 * t[u] + col - dd[v];
                if (jj >= 0 && jj < Jc) {
                    TQ *x = X + M::row(row, v) * xrow + jj;
                    *x = add ? *x + (TQ)acc[u][v] : (TQ)acc[u][v];
                }
            }
        }
    }
}

// LDS of the phased tile beyond its static arrays: coefficients
// [nd][KSP][64], then the chunk bins X [TS][xrow] and one 16-byte slot that
// takes the FP64 tiles' stores of bins outside the chunk (the prologue's
// scratch lives there first).
__host__ __device__ inline size_t ph_dyn_bytes(int ts, int nd, int nl, int wrow, size_t e)
{
    const size_t gb = (size_t)ts * wrow * e + 16;
    const size_t sb = prologue_scratch_bytes(ts, nd, nl);
    return coef_bytes<ENG_MFMA>(ts, nd, nl, e) + (gb > sb ? gb : sb);
}

// L phase of one chunk for one lane of the phased tile: the chunk's bins
// j0 + i, i = o, o + LPS, o + 2 LPS, ... < Jc, of its sample (o chosen by
// the caller so that the lane owns the bins j = sub (mod LPS) whatever the
// chunking), x = X[i] (the sum over the detectors), folded into the lane's
// log-sum-exp (m, s).  srow: the sample's series row at bin j0 when the
// per-bin values are wanted (minus q), else null.
template <typename TQ, int LPS, bool DUMP>
__device__ __forceinline__ void ph_lphase(const TQ *X, int Jc, int o, double &m, double &ssum,
                                          double *srow, double q)
{
    const auto xval = [&](int i) {
        const double x = (double)X[i];
        if (DUMP) srow[i] = x - q;
        return x;
    };
    // the terms e^d: FP64 tiles by exp_lse; FP32 tiles, whose bin values
    // carry FP32 rounding already, by the single-precision exponential (its
    // relative error, a few 1e-8, is below that of the values; the sums and
    // the reference stay FP64)
    const auto ex = [](double d) -> double {
        if constexpr (sizeof(TQ) == 4) return (double)expf((float)d);
        else return exp_lse(d);
    };
    const auto fold = [&](double x) {
        double d = x - m;
        if (d > kLseSlack) {
            ssum = m == -INFINITY ? 0.0 : ssum * exp(m - x);
            m = x;
            d = 0.0;
        }
        ssum += ex(d);
    };
    // two bins at a time: when neither moves the reference, their exps are
    // independent (the sums are still taken in bin order, as fold would)
    int i = o;
    for (; i + LPS < Jc; i += 2 * LPS) {
        const double x0 = xval(i), x1 = xval(i + LPS);
        const double d0 = x0 - m, d1 = x1 - m;
        if (d0 > kLseSlack || d1 > kLseSlack) {
            fold(x0);
            fold(x1);
        } else {
            const double e0 = ex(d0), e1 = ex(d1);
            ssum += e0;
            ssum += e1;
        }
    }
    if (i < Jc) fold(xval(i));
}

// PRE: the per-sample terms come from k_terms (the tile's block of the
// terms, tile-major from position t0), else the tile forms them
// (tile_prologue).
template <typename TQ, int TS, int NT, bool DUMP, bool PRE>
__device__ __forceinline__ void contract_tile_ph(
    const ile_geom &g, int64_t base, const double *__restrict__ smp, int64_t N,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ shifts,
    const TQ *__restrict__ Q, const double2 *__restrict__ U,
    const double2 *__restrict__ V, const double *__restrict__ terms, int64_t t0,
    double *__restrict__ out, double *__restrict__ series)
{
    static_assert(TS == 16 && (NT == 256 || NT == 512), "phased tile: 16 samples, 4 or 8 waves");
    constexpr int NW = NT / 64;    // waves
    constexpr int LPS = NT / TS;   // lanes per sample in the L phase
    __shared__ double s_q[TS];
    __shared__ int s_idx[TS], s_ok[TS];
    __shared__ int s_d[ILE_MAX_DET][TS];
    __shared__ int s_smin[ILE_MAX_DET], s_spread[ILE_MAX_DET];
    extern __shared__ __align__(16) unsigned char dyn_lds[];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nd = g.n_det, nl = g.n_lm, nq = g.n_q, n_t = g.n_t;
    const int KSP = ksp_of(nl), RP = 4 * KSP;
    const int wcap = g.wcap, wrow = g.wrow;
    TQ *coef = reinterpret_cast<TQ *>(dyn_lds);   // [nd][KSP][64]
    TQ *G = reinterpret_cast<TQ *>(dyn_lds + coef_bytes<ENG_MFMA>(TS, nd, nl, sizeof(TQ)));
    const size_t gbytes = (size_t)TS * wrow * sizeof(TQ);
    const size_t sbytes = prologue_scratch_bytes(TS, nd, nl);
    // one buffer resource over all of Q (the host keeps it below 2 GiB)
    const __amdgpu_buffer_rsrc_t rs = q_rsrc<TQ>(Q, nd * RP * nq * (int)sizeof(TQ));

    if constexpr (PRE) {
        // samples, validity, window starts and q of the tile; the
        // coefficients c = (d_ref/D) F_k Y_lm in the matrix-core A layout
        // (modes a in [nl, 2 KSP) are the zero padding of K)
        const double *tb = terms + ((base - t0) >> 4) * (16 * (int64_t)(2 + 3 * nd + 2 * nl));
        if (tid < TS) {
            const int64_t i = base + tid;
            int idx = -1, ok = 0;
            double q = 0.0;
            if (i < N) {
                const double *tk = tb + tid;
                idx = perm[i];
                ok = tk[16] != 0.0;
                q = tk[0];
                for (int k = 0; k < nd; k++) s_d[k][tid] = (int)tk[(2 + 2 * nd + 2 * nl + k) * 16];
            } else {
                for (int k = 0; k < nd; k++) s_d[k][tid] = 0;
            }
            s_idx[tid] = idx;
            s_ok[tid] = ok;
            s_q[tid] = q;
        }
        // the factors (d_ref/D) F_k and -2Y_lm of the tile's samples to LDS
        // (the free G blocks) in one round of loads, then the products
        double *s_fy = reinterpret_cast<double *>(G);   // [2 (nd + nl)][TS]
        const int nfy = 2 * (nd + nl);
        for (int t = tid; t < TS * nfy; t += NT)
            s_fy[t] = base + t % TS < N ? tb[2 * TS + t] : 0.0;
        __syncthreads();
        const int nlp = 2 * KSP;
        for (int t = tid; t < TS * nd * nlp; t += NT) {
            const int al = t % TS, r = t / TS, k = r / nlp, a = r - k * nlp;
            double cx = 0.0, cy = 0.0;
            if (a < nl) {
                const double fr = s_fy[(2 * k) * TS + al], fi = s_fy[(2 * k + 1) * TS + al];
                const double yr = s_fy[(2 * nd + 2 * a) * TS + al];
                const double yi = s_fy[(2 * nd + 2 * a + 1) * TS + al];
                cx = fr * yr - fi * yi;
                cy = fr * yi + fi * yr;
            }
            const int r0 = 2 * a;
            coef[(k * KSP + (r0 >> 2)) * 64 + (r0 & 3) * 16 + al] = (TQ)cx;
            coef[(k * KSP + (r0 >> 2)) * 64 + ((r0 & 3) + 1) * 16 + al] = (TQ)cy;
        }
        (void)gbytes;
        (void)sbytes;
        __syncthreads();
    } else {
        tile_prologue<TQ, TS, NT, ENG_MFMA>(g, base, smp, N, perm, shifts, U, V,
                                            reinterpret_cast<double *>(G),
                                            gbytes > sbytes ? gbytes : sbytes, coef, s_q,
                                            s_idx, s_ok, s_d);
    }

    // window range of each detector over the tile's valid samples
    if (tid < TS) {
        const bool v = s_ok[tid];
        for (int k = 0; k < nd; k++) {
            int lo = v ? s_d[k][tid] : 0x7fffffff, hi = v ? s_d[k][tid] : -1;
            for (int off = 8; off > 0; off >>= 1) {
                lo = min(lo, __shfl_xor(lo, off, 16));
                hi = max(hi, __shfl_xor(hi, off, 16));
            }
            if (tid == 0) {
                s_smin[k] = hi >= 0 ? lo : 0;
                s_spread[k] = hi >= 0 ? hi - lo : 0;
            }
        }
    }
    __syncthreads();

    using MA = mfma_acc<TQ>;
    // FP64 tiles store without branches (measured faster), the others with
    constexpr bool BF = sizeof(TQ) == 8 && !DUMP;
    const int al = tid / LPS, sub = tid % LPS, row = lane >> 4;
    const bool mem = s_ok[al];
    TQ *X = G;   // [TS][wrow], the chunk's bins of every sample
    double m = -INFINITY, ssum = 0.0;
    const int J = wcap;   // a multiple of 16, at most wrow
    for (int j0 = 0; j0 < n_t; j0 += J) {
        const int Jc = min(J, n_t - j0);
        // G phase, detector by detector: N-tiles wv, wv + NW, ..., four at
        // a time
        for (int k = 0; k < nd; k++) {
            const int smin = s_smin[k];
            const int T = (Jc + s_spread[k] + 15) >> 4;
            int dd[4];
#pragma unroll
            for (int v = 0; v < 4; v++) dd[v] = s_d[k][MA::row(row, v)] - smin;
            const TQ *coefk = coef + k * KSP * 64;
            for (int tb = wv; tb < T; tb += 4 * NW) {
                int t[4], nu = 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int tt = tb + u * NW;
                    t[u] = tt < T ? tt : tb;
                    nu += tt < T;
                }
                switch (__builtin_amdgcn_readfirstlane(nu)) {
                case 4: ph_tiles<TQ, 4, BF>(X, wrow, coefk, rs, k * RP, nq, KSP, smin + j0, t, dd, Jc, k > 0, lane); break;
                case 3: ph_tiles<TQ, 3, BF>(X, wrow, coefk, rs, k * RP, nq, KSP, smin + j0, t, dd, Jc, k > 0, lane); break;
                case 2: ph_tiles<TQ, 2, BF>(X, wrow, coefk, rs, k * RP, nq, KSP, smin + j0, t, dd, Jc, k > 0, lane); break;
                default: ph_tiles<TQ, 1, BF>(X, wrow, coefk, rs, k * RP, nq, KSP, smin + j0, t, dd, Jc, k > 0, lane); break;
                }
            }
            __syncthreads();
        }
        // L phase
        if (mem) {
            double *srow = DUMP ? series + (int64_t)s_idx[al] * n_t + j0 : nullptr;
            const int o = (sub - j0) & (LPS - 1);   // first bin j = sub (mod LPS)
            ph_lphase<TQ, LPS, DUMP>(X + al * wrow, Jc, o, m, ssum, srow, s_q[al]);
        }
        __syncthreads();
    }
    // merge the LPS lanes of each sample (fixed tree: 16-lane rows, then the
    // row pair), then the result (M - q) + log S - log n_t
    double M = row_max64(m);
    if (LPS == 32) M = fmax(M, __shfl_xor(M, 16));
    double S = row_sum64(m == -INFINITY ? 0.0 : ssum * exp(m - M));
    if (LPS == 32) S += __shfl_xor(S, 16);
    if (sub == 0 && s_idx[al] >= 0)
        out[s_idx[al]] = s_ok[al] ? (M - s_q[al]) + log(S) - log((double)n_t) : NAN;
}

template <typename TQ, int TS, int NT, int ENG, bool DUMP>
__device__ __forceinline__ void run_tile(
    const ile_geom &g, int64_t base, const double *__restrict__ smp, int64_t N,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ shifts,
    const TQ *__restrict__ Q, const double2 *__restrict__ U,
    const double2 *__restrict__ V, double *__restrict__ out,
    double *__restrict__ series)
{
    if constexpr (ENG == ENG_PH)
        contract_tile_ph<TQ, TS, NT, DUMP, false>(g, base, smp, N, perm, shifts, Q, U, V,
                                                  nullptr, 0, out, series);
    else
        contract_tile<TQ, TS, NT, ENG, DUMP>(g, base, smp, N, perm, shifts, Q, U, V, out, series);
}

// Waves per SIMD the register allocation must allow (the second bound of
// __launch_bounds__): two eight-wave phased workgroups per CU, as many as
// their LDS admits, are four waves per SIMD.
template <int NT, int ENG> constexpr int contract_min_waves() { return ENG == ENG_PH && NT == 512 ? 4 : 1; }

template <typename TQ, int TS, int NT, int ENG, bool DUMP>
__global__ __launch_bounds__(NT, (contract_min_waves<NT, ENG>())) void k_contract(
    ile_geom g, const double *__restrict__ smp, int64_t N,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ shifts,
    const TQ *__restrict__ Q, const double2 *__restrict__ U,
    const double2 *__restrict__ V, double *__restrict__ out,
    double *__restrict__ series)
{
    run_tile<TQ, TS, NT, ENG, DUMP>(g, (int64_t)blockIdx.x * TS, smp, N, perm, shifts,
                                    Q, U, V, out, series);
}

// Persistent form over many intrinsic points: every workgroup takes
// (point, tile) items from a queue in list order (the host sorts the list by
// decreasing cost) until it is empty; every wave reaches the exit.
template <typename TQ, int TS, int NT, int ENG>
__global__ __launch_bounds__(NT, (contract_min_waves<NT, ENG>())) void k_contract_batched(
    const ile_geom *__restrict__ geoms, const ile_point_dev *__restrict__ pts,
    const int2 *__restrict__ items, int n_items, unsigned *counter)
{
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // uniform, so the point's parameters load through the scalar unit
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 w = items[it];
        const ile_point_dev &P = pts[w.x];
        run_tile<TQ, TS, NT, ENG, false>(geoms[w.x], (int64_t)w.y * TS, P.smp, P.N,
                                         P.perm, P.shifts, (const TQ *)P.Q, P.U, P.V,
                                         P.out, nullptr);
    }
}

// Many intrinsic points on the phased engine: one workgroup per (point,
// tile) item, in list order (the host sorts the list by decreasing cost and
// the dispatcher starts workgroups in that order).  PRE: every point carries
// its per-sample terms; else the tiles form them.  Not persistent: every
// load of the point's parameters precedes the kernel's only store, so they
// are read through the scalar unit instead of being held in registers
// across a queue loop.
template <typename TQ, int TS, int NT, bool PRE>
__global__ __launch_bounds__(NT, (contract_min_waves<NT, ENG_PH>())) void k_contract_items(
    const ile_geom *__restrict__ geoms, const ile_point_dev *__restrict__ pts,
    const int2 *__restrict__ items)
{
    const int2 w = items[blockIdx.x];
    const ile_point_dev &P = pts[w.x];
    if (PRE)
        contract_tile_ph<TQ, TS, NT, false, true>(geoms[w.x], (int64_t)w.y * TS, P.smp, P.N,
                                                  P.perm, P.shifts, (const TQ *)P.Q, P.U, P.V,
                                                  P.terms, 0, P.out, nullptr);
    else
        contract_tile_ph<TQ, TS, NT, false, false>(geoms[w.x], (int64_t)w.y * TS, P.smp, P.N,
                                                   P.perm, P.shifts, (const TQ *)P.Q, P.U, P.V,
                                                   nullptr, 0, P.out, nullptr);
}

// One point on the phased engine with its per-sample terms precomputed:
// tiles of tile positions t0 + 16 blockIdx.x .. (below N), their terms
// tile-major from position t0.
template <typename TQ, int NT, bool DUMP>
__global__ __launch_bounds__(NT, (contract_min_waves<NT, ENG_PH>())) void k_contract_ph(
    ile_geom g, const double *__restrict__ smp, int64_t N, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ shifts, const TQ *__restrict__ Q,
    const double *__restrict__ terms, int64_t t0, double *__restrict__ out,
    double *__restrict__ series)
{
    contract_tile_ph<TQ, 16, NT, DUMP, true>(g, t0 + (int64_t)blockIdx.x * 16, smp, N, perm,
                                             shifts, Q, nullptr, nullptr, terms, t0, out,
                                             series);
}

// --------------------------------------------------------------- prior
using ile_rng::u53;

__global__ __launch_bounds__(256) void k_prior(uint64_t seed, int64_t first,
                                               int64_t N, double d_min,
                                               double d_max, double t_ref_max,
                                               double *smp, int64_t ld,
                                               double *ln_p)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const uint64_t i = (uint64_t)(first + t);
    uint32_t w[16];
    ile_rng::prior_words(seed, i, w);
    {
#pragma clang fp contract(off)
    const double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
    const double ra = 2.0 * kPi * u53(w[0], w[1]);
    const double dec = asin(2.0 * u53(w[2], w[3]) - 1.0);
    const double psi = kPi * u53(w[4], w[5]);
    const double phi = 2.0 * kPi * u53(w[6], w[7]);
    const double ci = 2.0 * u53(w[8], w[9]) - 1.0;
    const double D = cbrt(d_min * d_min * d_min + u53(w[10], w[11]) * v3);
    const double tr = t_ref_max * (2.0 * u53(w[12], w[13]) - 1.0);
    smp[0 * ld + t] = ra;
    smp[1 * ld + t] = dec;
    smp[2 * ld + t] = psi;
    smp[3 * ld + t] = phi;
    smp[4 * ld + t] = ci;
    smp[5 * ld + t] = D;
    smp[6 * ld + t] = tr;
    if (ln_p)
        ln_p[t] = -log(kTwoPi) + log(cos(dec) / 2.0) - log(kPi) - log(kTwoPi) -
                  log(2.0) + log(3.0 * D * D / v3) - log(2.0 * t_ref_max);
    }
}

// ------------------------------------------------------------- reduction
constexpr int kRedBlocks = 256;
constexpr int kRedT = 256;

__device__ inline double lnw_at(const double *lnL, const double *lp,
                                const double *lq, int64_t i)
{
    return lnL[i] + (lp ? lp[i] : 0.0) - (lq ? lq[i] : 0.0);
}

__global__ __launch_bounds__(kRedT) void k_red_max(const double *lnL,
                                                   const double *lp,
                                                   const double *lq, int64_t N,
                                                   double *tmp)
{
    __shared__ double sm[kRedT], sl[kRedT];
    double M = -INFINITY, ML = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kRedT + threadIdx.x; i < N;
         i += (int64_t)kRedBlocks * kRedT) {
        double w = lnw_at(lnL, lp, lq, i);
        M = w > M ? w : M;
        ML = lnL[i] > ML ? lnL[i] : ML;
    }
    sm[threadIdx.x] = M;
    sl[threadIdx.x] = ML;
    __syncthreads();
    for (int s = kRedT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
            sl[threadIdx.x] = fmax(sl[threadIdx.x], sl[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tmp[blockIdx.x] = sm[0];
        tmp[kRedBlocks + blockIdx.x] = sl[0];
    }
}

__device__ inline double global_max(const double *tmp)
{
    double M = -INFINITY;
    for (int b = 0; b < kRedBlocks; b++) M = fmax(M, tmp[b]);
    return M;
}

__global__ __launch_bounds__(kRedT) void k_red_sum(const double *lnL,
                                                   const double *lp,
                                                   const double *lq, int64_t N,
                                                   double *tmp)
{
    __shared__ double s1[kRedT], s2[kRedT];
    __shared__ double sM;
    if (threadIdx.x == 0) sM = global_max(tmp);
    __syncthreads();
    const double M = sM;
    double a = 0.0, b = 0.0;
    if (M != -INFINITY) {
        for (int64_t i = (int64_t)blockIdx.x * kRedT + threadIdx.x; i < N;
             i += (int64_t)kRedBlocks * kRedT) {
            double e = exp(lnw_at(lnL, lp, lq, i) - M);
            a += e;
            b += e * e;
        }
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int s = kRedT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tmp[2 * kRedBlocks + blockIdx.x] = s1[0];
        tmp[3 * kRedBlocks + blockIdx.x] = s2[0];
    }
}

__global__ __launch_bounds__(kRedT) void k_red_final(const double *tmp,
                                                     int64_t N, double *partial)
{
    __shared__ double s1[kRedT], s2[kRedT], sl[kRedT];
    const int t = threadIdx.x;   // kRedT == kRedBlocks
    s1[t] = tmp[2 * kRedBlocks + t];
    s2[t] = tmp[3 * kRedBlocks + t];
    sl[t] = tmp[kRedBlocks + t];
    __syncthreads();
    for (int s = kRedT / 2; s > 0; s >>= 1) {
        if (t < s) {
            s1[t] += s1[t + s];
            s2[t] += s2[t + s];
            sl[t] = fmax(sl[t], sl[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        partial[0] = global_max(tmp);
        partial[1] = s1[0];
        partial[2] = s2[0];
        partial[3] = (double)N;
        partial[4] = sl[0];
    }
}

// The same partial from one workgroup when N is small (at most
// kRedSmallMax): the three kernels above cost more in launches and in their
// mostly idle blocks than the work.  Same quantities, its own summation tree.
constexpr int kRedSmallT = 1024;
constexpr int64_t kRedSmallMax = 16384;

__global__ __launch_bounds__(kRedSmallT) void k_red_small(const double *lnL, const double *lp,
                                                           const double *lq, int64_t N,
                                                           double *partial)
{
    __shared__ double sa[kRedSmallT], sb[kRedSmallT], sc[kRedSmallT];
    const int t = threadIdx.x;
    double M = -INFINITY, ML = -INFINITY;
    for (int64_t i = t; i < N; i += kRedSmallT) {
        const double w = lnw_at(lnL, lp, lq, i);
        M = w > M ? w : M;
        ML = lnL[i] > ML ? lnL[i] : ML;
    }
    sa[t] = M;
    sc[t] = ML;
    __syncthreads();
    for (int h = kRedSmallT / 2; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] = fmax(sa[t], sa[t + h]);
            sc[t] = fmax(sc[t], sc[t + h]);
        }
        __syncthreads();
    }
    const double Mg = sa[0];
    __syncthreads();
    double a = 0.0, b = 0.0;
    if (Mg != -INFINITY) {
        for (int64_t i = t; i < N; i += kRedSmallT) {
            const double e = exp(lnw_at(lnL, lp, lq, i) - Mg);
            a += e;
            b += e * e;
        }
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = kRedSmallT / 2; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        partial[0] = Mg;
        partial[1] = sa[0];
        partial[2] = sb[0];
        partial[3] = (double)N;
        partial[4] = sc[0];
    }
}

__global__ void k_finish(const double *parts, int n_part, double *res)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double M = -INFINITY, ML = -INFINITY, n = 0.0;
    for (int i = 0; i < n_part; i++) {
        M = fmax(M, parts[5 * i]);
        ML = fmax(ML, parts[5 * i + 4]);
        n += parts[5 * i + 3];
    }
    double S1 = 0.0, S2 = 0.0;
    if (M != -INFINITY)
        for (int i = 0; i < n_part; i++) {
            if (parts[5 * i] == -INFINITY) continue;
            double e = exp(parts[5 * i] - M);
            S1 += parts[5 * i + 1] * e;
            S2 += parts[5 * i + 2] * e * e;
        }
    if (M == -INFINITY || n == 0.0) {
        res[0] = -INFINITY;
        res[1] = 0.0;
        res[2] = 0.0;
        res[3] = NAN;
    } else {
        res[0] = M + log(S1) - log(n);
        res[1] = S1;
        res[2] = S1 * S1 / S2;
        double var = S2 / (S1 * S1) - 1.0 / n;
        res[3] = var > 0.0 ? sqrt(var) : 0.0;
    }
    res[4] = ML;
    res[5] = n;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename TQ, int TS, int NT, int ENG>
hipError_t launch_contract_t(const ile_geom &g, const double *smp, int64_t N,
                             const int32_t *perm, const int32_t *shifts,
                             const void *Q, const double *U, const double *V,
                             double *out, double *series, hipStream_t st)
{
    size_t dyn = coef_bytes<ENG>(TS, g.n_det, g.n_lm, sizeof(TQ));
    const size_t scr = prologue_scratch_bytes(TS, g.n_det, g.n_lm);
    if (scr > (size_t)TS * NT * sizeof(TQ)) dyn += scr;
    const unsigned grid = nblk(N, TS);
    if (series)
        hipLaunchKernelGGL((k_contract<TQ, TS, NT, ENG, true>), dim3(grid), dim3(NT), dyn, st,
                           g, smp, N, perm, shifts, (const TQ *)Q,
                           (const double2 *)U, (const double2 *)V, out, series);
    else
        hipLaunchKernelGGL((k_contract<TQ, TS, NT, ENG, false>), dim3(grid), dim3(NT), dyn, st,
                           g, smp, N, perm, shifts, (const TQ *)Q,
                           (const double2 *)U, (const double2 *)V, out, series);
    return hipGetLastError();
}

// Bins per chunk of the phased engine (also the LDS row stride of its bin
// rows): the largest that keeps the workgroup's dynamic LDS within `budget`
// bytes, an odd multiple of 128 bytes so that rows of neighbouring samples
// start in alternate halves of the 256-byte bank period.  0 if none fits.
int ph_wrow(int nd, int nl, size_t e, size_t budget)
{
    const size_t fixed = coef_bytes<ENG_MFMA>(16, nd, nl, e) + 16;   // + the slot past X
    if (budget <= fixed) return 0;
    const int unit = (int)(128 / e);
    const int w = (int)((budget - fixed) / ((size_t)16 * e));
    const int q = (w / unit - 1) / 2;
    return q < 0 ? 0 : unit * (2 * q + 1);
}

// Default LDS budgets of a phased workgroup: FP64 tiles hold four waves per
// SIMD in registers, two workgroups per CU; FP32 tiles need fewer registers
// and run three per CU.
constexpr size_t kPhBudget64 = 78 * 1024;
constexpr size_t kPhBudget32 = 50 * 1024;

static hipError_t launch_terms(const ile_geom &g, const double *smp, int64_t N,
                               const int32_t *perm, const int32_t *shifts, bool in_order,
                               const double4 *uvt, int64_t t0, int64_t n, double *terms,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_terms, dim3(nblk(n, kTermsT)), dim3(kTermsT), terms_lds_bytes(g), st,
                       g, smp, N, perm, shifts, in_order, uvt, t0, n, terms);
    return hipGetLastError();
}

// Raises kernel fn's dynamic LDS limit on the current device to at least
// dyn bytes (never lowers it: another thread may launch with a larger
// size).  allowed: the kernel's per-device record of what was set.
static hipError_t allow_dyn_lds(const void *fn, size_t dyn, size_t (&allowed)[64])
{
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (dyn <= allowed[dev]) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e == hipSuccess) allowed[dev] = dyn;
    return e;
}

template <typename TQ, int NT, bool DUMP>
hipError_t launch_contract_ph(const ile_geom &g, const double *smp, int64_t N,
                              const int32_t *perm, const int32_t *shifts, const double *smp_s,
                              const int32_t *sh_s, const void *Q, const double4 *uvt,
                              double *terms, int64_t cap, double *out, double *series, size_t dyn,
                              hipStream_t st)
{
    // dynamic LDS above the default limit must be allowed per kernel
    static size_t allowed[64] = {};
    hipError_t ea = allow_dyn_lds(reinterpret_cast<const void *>(&k_contract_ph<TQ, NT, DUMP>),
                                  dyn, allowed);
    if (ea != hipSuccess) return ea;
    for (int64_t t0 = 0; t0 < N; t0 += cap) {
        const int64_t n = N - t0 < cap ? N - t0 : cap;
        hipError_t e = smp_s ? launch_terms(g, smp_s, N, perm, sh_s, true, uvt, t0, n, terms, st)
                             : launch_terms(g, smp, N, perm, shifts, false, uvt, t0, n, terms, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_contract_ph<TQ, NT, DUMP>), dim3(nblk(n, 16)), dim3(NT), dyn, st, g,
                           smp, N, perm, shifts, (const TQ *)Q, (const double *)terms, t0, out,
                           series);
    }
    return hipGetLastError();
}

// Allows the persistent phased kernel `dyn` bytes of dynamic LDS (outside
// any stream capture: the batch calls it before capturing its graph).
template <typename TQ, int NT>
hipError_t allow_batched_ph(size_t dyn)
{
    static size_t allowed[64] = {}, allowed_pre[64] = {};
    hipError_t e = allow_dyn_lds(reinterpret_cast<const void *>(&k_contract_items<TQ, 16, NT, false>),
                                 dyn, allowed);
    if (e != hipSuccess) return e;
    return allow_dyn_lds(reinterpret_cast<const void *>(&k_contract_items<TQ, 16, NT, true>), dyn,
                         allowed_pre);
}

template <typename TQ, int NT>
hipError_t launch_batched_ph(const ile_geom *geoms, const ile_point_dev *pts, const int2 *items,
                             int n_items, size_t dyn, bool pre, hipStream_t st)
{
    hipError_t e = allow_batched_ph<TQ, NT>(dyn);
    if (e != hipSuccess) return e;
    // a dispatch covers fewer than 2^32 work-items: at most 2^22 items each
    constexpr int kMaxItems = 1 << 22;
    for (int i0 = 0; i0 < n_items; i0 += kMaxItems) {
        const int n = n_items - i0 < kMaxItems ? n_items - i0 : kMaxItems;
        if (pre)
            hipLaunchKernelGGL((k_contract_items<TQ, 16, NT, true>), dim3((unsigned)n), dim3(NT),
                               dyn, st, geoms, pts, items + i0);
        else
            hipLaunchKernelGGL((k_contract_items<TQ, 16, NT, false>), dim3((unsigned)n), dim3(NT),
                               dyn, st, geoms, pts, items + i0);
    }
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t ile_launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t ile_launch_prep(const ile_geom &g, const double *smp, int64_t N,
                           int32_t *shifts, uint32_t *keys, uint32_t *hist,
                           uint32_t n_buckets, int32_t *err, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3(nblk(N, 256)), dim3(256), 0, st, g, smp, N,
                       shifts, keys, hist, n_buckets, err);
    return hipGetLastError();
}

int64_t ile_scan_tmp_words(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t ile_launch_scan(uint32_t *v, int64_t n, uint32_t *tmp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = ile_scan_tmp_words(n);
    if (nb > kScanBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanT), 0, st, v, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanT), 0, st, tmp, (int)nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n, 256)), dim3(256), 0, st, v, n,
                       (const uint32_t *)tmp);
    return hipGetLastError();
}

hipError_t ile_launch_scatter(const uint32_t *keys, int64_t N, uint32_t *offs,
                              int32_t *perm, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(nblk(N, 256)), dim3(256), 0, st, keys, N,
                       offs, perm);
    return hipGetLastError();
}

hipError_t ile_launch_scatter_copy(const uint32_t *keys, int64_t N, uint32_t *offs,
                                   int32_t *perm, const double *smp, const int32_t *shifts,
                                   int nd, double *smp_s, int32_t *sh_s, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_copy, dim3(nblk(N, 256)), dim3(256), 0, st, keys, N, offs, perm,
                       smp, shifts, nd, smp_s, sh_s);
    return hipGetLastError();
}

hipError_t ile_launch_identity(int32_t *perm, int64_t N, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_identity, dim3(nblk(N, 256)), dim3(256), 0, st, perm, N);
    return hipGetLastError();
}

static int kernel_threads(const ile_tune &tu)
{
    return tu.engine == ENG_MFMA ? 2 * tu.threads : tu.threads;
}

static size_t ph_budget(const ile_tune &tu, size_t e)
{
    if (tu.lds_budget > 0) return (size_t)tu.lds_budget;
    return e == 8 ? kPhBudget64 : kPhBudget32;
}

void ile_contract_prepare(ile_geom &g, ile_precision prec, const ile_tune &tu)
{
    if (tu.engine == ENG_PH && prec != ILE_BF16) {
        const size_t e = prec == ILE_FP64 ? 8 : 4;
        g.wrow = g.wcap = ph_wrow(g.n_det, g.n_lm, e, ph_budget(tu, e));
    } else {
        g.wrow = g.wcap = 0;
    }
}

static size_t coef_bytes_of(const ile_geom &g, ile_precision prec, const ile_tune &tu, size_t e)
{
    if (prec == ILE_BF16) return coef_bytes<ENG_BF16>(tu.tile_samples, g.n_det, g.n_lm, e);
    return tu.engine == ENG_MFMA ? coef_bytes<ENG_MFMA>(tu.tile_samples, g.n_det, g.n_lm, e)
                                 : coef_bytes<ENG_VALU>(tu.tile_samples, g.n_det, g.n_lm, e);
}

size_t ile_contract_lds_bytes(const ile_geom &g, ile_precision prec,
                              const ile_tune &tu)
{
    const size_t e = prec == ILE_FP64 ? 8 : 4;
    if (tu.engine == ENG_PH && prec != ILE_BF16) {
        const int w = ph_wrow(g.n_det, g.n_lm, e, ph_budget(tu, e));
        // a chunk has at least 16 bins
        if (w < 16) return (size_t)1 << 30;
        return ph_dyn_bytes(16, g.n_det, g.n_lm, w, e) + 2048;
    }
    const size_t gs = (size_t)tu.tile_samples * (tu.engine == ENG_MFMA ? 2 : 1) * tu.threads * e;
    const size_t coef = coef_bytes_of(g, prec, tu, e);
    const size_t scr = prologue_scratch_bytes(tu.tile_samples, g.n_det, g.n_lm);
    return gs + coef + (scr > gs ? scr : 0) + 4096;
}

bool ile_tune_supported(ile_precision prec, const ile_tune &tu)
{
    if (tu.tile_samples != 16) return false;
    // the phased engine takes FP64 and FP32 operands in workgroups of four
    // or eight waves; its block width follows from the LDS budget
    if (tu.engine == ENG_PH) return prec != ILE_BF16 && (tu.threads == 256 || tu.threads == 512);
    // positions per block: 256 or 512 for both engines; the matrix-core
    // engines also take 128 and 192 (smaller LDS, more workgroups per CU)
    const bool mf_only = tu.threads == 128 || tu.threads == 192;
    if (tu.threads != 256 && tu.threads != 512 && !mf_only) return false;
    if (prec == ILE_BF16) return tu.engine == ENG_MFMA;   // BF16 runs on the matrix cores only
    if (mf_only) return tu.engine == ENG_MFMA;
    return tu.engine == ENG_MFMA || tu.engine == ENG_VALU;
}

int ile_terms_fields(const ile_geom &g) { return 2 + 3 * g.n_det + 2 * g.n_lm; }

hipError_t ile_launch_terms(const ile_geom &g, const double *smp, int64_t N,
                            const int32_t *perm, const int32_t *shifts, const double *uvt,
                            double *terms, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    if (terms_lds_bytes(g) > 64 * 1024) return hipErrorInvalidValue;
    return launch_terms(g, smp, N, perm, shifts, false, (const double4 *)uvt, 0, N, terms, st);
}

bool ile_contract_uses_terms(ile_precision prec, const ile_tune &tu)
{
    return tu.engine == ENG_PH && prec != ILE_BF16;
}

hipError_t ile_launch_contract(const ile_geom &g, ile_precision prec,
                               const ile_tune &tu, const double *smp, int64_t N,
                               const int32_t *perm, const int32_t *shifts,
                               const void *Q, const double *U, const double *V,
                               const double *smp_s, const int32_t *sh_s, const double *uvt,
                               double *terms, int64_t cap, double *out, double *series,
                               hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    if (!ile_tune_supported(prec, tu)) return hipErrorInvalidValue;
    if (tu.engine == ENG_PH) {
        ile_geom gp = g;
        ile_contract_prepare(gp, prec, tu);
        if (gp.wcap < 16) return hipErrorInvalidValue;
        if (!uvt || !terms || cap < 16 || cap % 16) return hipErrorInvalidValue;
        if (terms_lds_bytes(g) > 64 * 1024) return hipErrorInvalidValue;
        const size_t e = prec == ILE_FP64 ? 8 : 4;
        // one 32-bit buffer range covers the whole series
        if ((size_t)g.n_det * 4 * ksp_of(g.n_lm) * g.n_q * e > 0x7fffffffu)
            return hipErrorInvalidValue;
        const size_t dyn = ph_dyn_bytes(16, g.n_det, g.n_lm, gp.wrow, e);
#define ILE_PH(TQ, NT)                                                                       \
    return series ? launch_contract_ph<TQ, NT, true>(gp, smp, N, perm, shifts, smp_s, sh_s, Q,  \
                                                     (const double4 *)uvt, terms, cap, out,    \
                                                     series, dyn, st)                          \
                  : launch_contract_ph<TQ, NT, false>(gp, smp, N, perm, shifts, smp_s, sh_s,   \
                                                      Q, (const double4 *)uvt, terms, cap,     \
                                                      out, series, dyn, st)
        if (prec == ILE_FP64) {
            if (tu.threads == 256) ILE_PH(double, 256);
            ILE_PH(double, 512);
        }
        if (tu.threads == 256) ILE_PH(float, 256);
        ILE_PH(float, 512);
#undef ILE_PH
    }
#define ILE_CONTRACT(TQ, NT, ENG) \
    return launch_contract_t<TQ, 16, NT, ENG>(g, smp, N, perm, shifts, Q, U, V, out, series, st)
    if (prec == ILE_FP64) {
        if (tu.engine == ENG_MFMA) {
            // producer + consumer halves: threads = 2 x positions per block
            if (tu.threads == 512) ILE_CONTRACT(double, 1024, ENG_MFMA);
            if (tu.threads == 192) ILE_CONTRACT(double, 384, ENG_MFMA);
            if (tu.threads == 128) ILE_CONTRACT(double, 256, ENG_MFMA);
            ILE_CONTRACT(double, 512, ENG_MFMA);
        }
        if (tu.threads == 512) ILE_CONTRACT(double, 512, ENG_VALU);
        ILE_CONTRACT(double, 256, ENG_VALU);
    }
    if (prec == ILE_BF16) {
        if (tu.threads == 512) ILE_CONTRACT(float, 1024, ENG_BF16);
        if (tu.threads == 192) ILE_CONTRACT(float, 384, ENG_BF16);
        if (tu.threads == 128) ILE_CONTRACT(float, 256, ENG_BF16);
        ILE_CONTRACT(float, 512, ENG_BF16);
    }
    if (tu.engine == ENG_MFMA) {
        if (tu.threads == 512) ILE_CONTRACT(float, 1024, ENG_MFMA);
        if (tu.threads == 192) ILE_CONTRACT(float, 384, ENG_MFMA);
        if (tu.threads == 128) ILE_CONTRACT(float, 256, ENG_MFMA);
        ILE_CONTRACT(float, 512, ENG_MFMA);
    }
    if (tu.threads == 512) ILE_CONTRACT(float, 512, ENG_VALU);
    ILE_CONTRACT(float, 256, ENG_VALU);
#undef ILE_CONTRACT
}

size_t ile_contract_dyn_bytes(const ile_geom &g, ile_precision prec, const ile_tune &tu)
{
    const size_t e = prec == ILE_FP64 ? 8 : 4;
    if (tu.engine == ENG_PH && prec != ILE_BF16)
        return ph_dyn_bytes(16, g.n_det, g.n_lm, ph_wrow(g.n_det, g.n_lm, e, ph_budget(tu, e)), e);
    size_t dyn = coef_bytes_of(g, prec, tu, e);
    const size_t scr = prologue_scratch_bytes(tu.tile_samples, g.n_det, g.n_lm);
    if (scr > (size_t)tu.tile_samples * kernel_threads(tu) * e) dyn += scr;
    return dyn;
}

hipError_t ile_contract_batched_allow(ile_precision prec, const ile_tune &tu, size_t dyn)
{
    if (tu.engine != ENG_PH || prec == ILE_BF16) return hipSuccess;
    if (prec == ILE_FP64)
        return tu.threads == 256 ? allow_batched_ph<double, 256>(dyn)
                                 : allow_batched_ph<double, 512>(dyn);
    return tu.threads == 256 ? allow_batched_ph<float, 256>(dyn) : allow_batched_ph<float, 512>(dyn);
}

hipError_t ile_launch_contract_batched(ile_precision prec, const ile_tune &tu,
                                       const ile_geom *geoms, const ile_point_dev *pts,
                                       const int2 *items, int n_items, unsigned *counter,
                                       int grid, size_t dyn, bool terms, hipStream_t st)
{
    if (!ile_tune_supported(prec, tu)) return hipErrorInvalidValue;
    if (tu.engine == ENG_PH) {
        // one workgroup per item (grid and counter are for the persistent
        // kernels of the other engines)
        if (prec == ILE_FP64)
            return tu.threads == 256
                       ? launch_batched_ph<double, 256>(geoms, pts, items, n_items, dyn, terms, st)
                       : launch_batched_ph<double, 512>(geoms, pts, items, n_items, dyn, terms, st);
        return tu.threads == 256
                   ? launch_batched_ph<float, 256>(geoms, pts, items, n_items, dyn, terms, st)
                   : launch_batched_ph<float, 512>(geoms, pts, items, n_items, dyn, terms, st);
    }
#define ILE_BATCHED(TQ, NT, ENG)                                                              \
    do {                                                                                      \
        hipLaunchKernelGGL((k_contract_batched<TQ, 16, NT, ENG>), dim3(grid), dim3(NT), dyn,   \
                           st, geoms, pts, items, n_items, counter);                          \
        return hipGetLastError();                                                             \
    } while (0)
    if (prec == ILE_FP64) {
        if (tu.engine == ENG_MFMA) {
            if (tu.threads == 512) ILE_BATCHED(double, 1024, ENG_MFMA);
            if (tu.threads == 192) ILE_BATCHED(double, 384, ENG_MFMA);
            if (tu.threads == 128) ILE_BATCHED(double, 256, ENG_MFMA);
            ILE_BATCHED(double, 512, ENG_MFMA);
        }
        if (tu.threads == 512) ILE_BATCHED(double, 512, ENG_VALU);
        ILE_BATCHED(double, 256, ENG_VALU);
    }
    if (prec == ILE_BF16) {
        if (tu.threads == 512) ILE_BATCHED(float, 1024, ENG_BF16);
        if (tu.threads == 192) ILE_BATCHED(float, 384, ENG_BF16);
        if (tu.threads == 128) ILE_BATCHED(float, 256, ENG_BF16);
        ILE_BATCHED(float, 512, ENG_BF16);
    }
    if (tu.engine == ENG_MFMA) {
        if (tu.threads == 512) ILE_BATCHED(float, 1024, ENG_MFMA);
        if (tu.threads == 192) ILE_BATCHED(float, 384, ENG_MFMA);
        if (tu.threads == 128) ILE_BATCHED(float, 256, ENG_MFMA);
        ILE_BATCHED(float, 512, ENG_MFMA);
    }
    if (tu.threads == 512) ILE_BATCHED(float, 512, ENG_VALU);
    ILE_BATCHED(float, 256, ENG_VALU);
#undef ILE_BATCHED
}

hipError_t ile_launch_prior(uint64_t seed, int64_t first, int64_t N,
                            double d_min, double d_max, double t_ref_max,
                            double *smp, int64_t ld, double *ln_p, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prior, dim3(nblk(N, 256)), dim3(256), 0, st, seed, first,
                       N, d_min, d_max, t_ref_max, smp, ld, ln_p);
    return hipGetLastError();
}

int ile_reduce_blocks() { return kRedBlocks; }

hipError_t ile_launch_reduce(const double *lnL, const double *ln_p,
                             const double *ln_q, int64_t N, double *tmp,
                             double *partial, hipStream_t st)
{
    if (N <= kRedSmallMax) {
        hipLaunchKernelGGL(k_red_small, dim3(1), dim3(kRedSmallT), 0, st, lnL, ln_p, ln_q, N,
                           partial);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_red_max, dim3(kRedBlocks), dim3(kRedT), 0, st, lnL, ln_p,
                       ln_q, N, tmp);
    hipLaunchKernelGGL(k_red_sum, dim3(kRedBlocks), dim3(kRedT), 0, st, lnL, ln_p,
                       ln_q, N, tmp);
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kRedT), 0, st, (const double *)tmp,
                       N, partial);
    return hipGetLastError();
}

hipError_t ile_launch_finish(const double *partials, int n_part, double *result,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, partials, n_part, result);
    return hipGetLastError();
}

hipError_t ile_launch_to_bf16_split(const double *, int64_t, void *, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t ile_launch_inject(const ile_geom &g, const double *h, int n, const double *theta,
                             double *d, hipStream_t st)
{
    const int64_t tot = (int64_t)g.n_det * n;
    hipLaunchKernelGGL(k_inject_resp, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g,
                       (const double2 *)h, n, theta, d);
    return hipGetLastError();
}

hipError_t ile_launch_inject_qv(int n_det, int n_lm, int n, const double *h, const double *d,
                                double scale, double *Q, double *U, double *V, hipStream_t st)
{
    hipLaunchKernelGGL(k_inject_corr, dim3((unsigned)((n + 255) / 256), (unsigned)(n_det * n_lm)),
                       dim3(256), 0, st, n_lm, n, (const double2 *)h, d, scale, (double2 *)Q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inject_gram, dim3((unsigned)(n_lm * n_lm)), dim3(256), 0, st, n_lm, n,
                       (const double2 *)h, (double2 *)U, (double2 *)V);
    return hipGetLastError();
}
