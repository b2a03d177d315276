// ile_sampler.hip -- device samplers of the Monte Carlo over extrinsic
// parameters (arXiv:1902.04934, Sec. II.A: direct Monte Carlo with an
// adaptive sampling prior; Sec. III.B: the sampling prior is regenerated
// from the most recent chunk of points, in the two sky parameters).
//
// The adaptive proposal is a product of two nb-bin histogram densities, in
// ra on [0, 2 pi) and in sin(dec) on [-1, 1], times the prior in psi, phi,
// cos(iota), D and t_ref.  Draws use the counter-based Philox stream of the
// prior draw; ra and sin(dec) go through the inverse CDF of the histograms.
// Refits temper the chunk's weights, w = exp(beta (ln w - max)),
// beta = min(1, scale / (max - mean)), sum them per bin and mix the result
// with the prior: P = (1 - floor) H / sum H + floor / nb.  Every sum runs in
// a fixed order, so a refit is bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ile_internal.h"
#include "ile_rng.h"

namespace {


using ile_rng::u53;

constexpr int kMaxBins = 64;   // per-thread LDS histograms: 64 threads x 2 x 64 doubles = 64 KB

__global__ __launch_bounds__(256) void k_hist_draw(
    uint64_t seed, int64_t first, int64_t N, int nb, const double *__restrict__ P,
    const double *__restrict__ C, double d_min, double d_max, double t_ref_max,
    double *smp, int64_t ld, double *ln_p, double *ln_q, int32_t *bins)
{
    __shared__ double sP[2 * kMaxBins], sC[2 * (kMaxBins + 1)];
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) sP[i] = P[i];
    for (int i = threadIdx.x; i < 2 * (nb + 1); i += blockDim.x) sC[i] = C[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const uint64_t i = (uint64_t)(first + t);
    uint32_t w[16];
    ile_rng::prior_words(seed, i, w);
    double x[7];
    int br, bs;
    const double lp = ile_rng::hist_sample(sP, sC, nb, w, d_min, d_max, t_ref_max, x, br, bs);
    for (int d = 0; d < 7; d++) smp[d * ld + t] = x[d];
    if (ln_p) ln_p[t] = lp;
    if (ln_q) ln_q[t] = lp + log(nb * sP[br]) + log(nb * sP[nb + bs]);
    if (bins) {
        bins[t] = br;
        bins[ld + t] = bs;
    }
}

__device__ inline double lnw_of(const double *lnL, const double *lp, const double *lq,
                                int64_t i)
{
    return lnL[i] + (lp ? lp[i] : 0.0) - (lq ? lq[i] : 0.0);
}

constexpr int kStatBlocks = 128, kStatT = 256;

// per-block max and sum of ln w
__global__ __launch_bounds__(kStatT) void k_lnw_stats(const double *lnL, const double *lp,
                                                      const double *lq, int64_t N,
                                                      double *part)
{
    __shared__ double sm[kStatT], ss[kStatT];
    double M = -INFINITY, S = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kStatT + threadIdx.x; i < N;
         i += (int64_t)kStatBlocks * kStatT) {
        const double v = lnw_of(lnL, lp, lq, i);
        M = fmax(M, v);
        S += v;
    }
    sm[threadIdx.x] = M;
    ss[threadIdx.x] = S;
    __syncthreads();
    for (int s = kStatT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
            ss[threadIdx.x] += ss[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sm[0];
        part[2 * blockIdx.x + 1] = ss[0];
    }
}

// beta and the max, from the per-block partials (fixed order)
__global__ void k_lnw_beta(const double *part, int64_t N, double scale, double *stats)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double M = -INFINITY, S = 0.0;
    for (int b = 0; b < kStatBlocks; b++) {
        M = fmax(M, part[2 * b]);
        S += part[2 * b + 1];
    }
    const double mean = S / (double)N;
    stats[0] = M;
    stats[1] = (M - mean) > scale ? scale / (M - mean) : 1.0;
}

constexpr int kHistT = 64;   // threads per block, each with private histograms

// per-thread private bin sums in LDS over a contiguous range per block, then
// a fixed-order sum over the block's threads
__global__ __launch_bounds__(kHistT) void k_hist_partial(
    const int32_t *__restrict__ bins, int64_t ld, const double *lnL, const double *lp,
    const double *lq, int64_t N, int nb, int64_t per_block, const double *stats,
    double *part)
{
    extern __shared__ double H[];   // [kHistT][2 nb]
    const int t = threadIdx.x;
    for (int b = 0; b < 2 * nb; b++) H[t * 2 * nb + b] = 0.0;
    const double M = stats[0], beta = stats[1];
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(lo + per_block, N);
    for (int64_t i = lo + t; i < hi; i += kHistT) {
        const double w = exp(beta * (lnw_of(lnL, lp, lq, i) - M));
        H[t * 2 * nb + bins[i]] += w;
        H[t * 2 * nb + nb + bins[ld + i]] += w;
    }
    __syncthreads();
    for (int b = t; b < 2 * nb; b += kHistT) {
        double s = 0.0;
        for (int u = 0; u < kHistT; u++) s += H[u * 2 * nb + b];
        part[(int64_t)blockIdx.x * 2 * nb + b] = s;
    }
}

// new histograms: fixed-order sum of the block partials, normalization,
// prior floor, cumulative sums
__global__ void k_hist_finish(const double *part, int nblk, int nb, double floor_w,
                              double *P, double *C)
{
    __shared__ double sH[2 * kMaxBins];
    for (int b = threadIdx.x; b < 2 * nb; b += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nblk; k++) s += part[(int64_t)k * 2 * nb + b];
        sH[b] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int h = threadIdx.x;
        double tot = 0.0;
        for (int b = 0; b < nb; b++) tot += sH[h * nb + b];
        double c = 0.0;
        C[h * (nb + 1)] = 0.0;
        for (int b = 0; b < nb; b++) {
            const double p = (1.0 - floor_w) * (sH[h * nb + b] / tot) + floor_w / nb;
            P[h * nb + b] = p;
            c += p;
            C[h * (nb + 1) + b + 1] = c;
        }
    }
}

// uniform histograms (the prior) and their cumulative sums
__global__ void k_hist_uniform(int nb, double *P, double *C)
{
    if (threadIdx.x < 2 && blockIdx.x == 0) {
        const int h = threadIdx.x;
        double c = 0.0;
        C[h * (nb + 1)] = 0.0;
        for (int b = 0; b < nb; b++) {
            P[h * nb + b] = 1.0 / nb;
            c += 1.0 / nb;
            C[h * (nb + 1) + b + 1] = c;
        }
    }
}

// cumulative sums of given histograms
__global__ void k_hist_cdf(int nb, const double *P, double *C)
{
    if (threadIdx.x < 2 && blockIdx.x == 0) {
        const int h = threadIdx.x;
        double c = 0.0;
        C[h * (nb + 1)] = 0.0;
        for (int b = 0; b < nb; b++) {
            c += P[h * nb + b];
            C[h * (nb + 1) + b + 1] = c;
        }
    }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int ile_hist_max_bins() { return kMaxBins; }

hipError_t ile_launch_hist_uniform(int nb, double *P, double *C, hipStream_t st)
{
    hipLaunchKernelGGL(k_hist_uniform, dim3(1), dim3(64), 0, st, nb, P, C);
    return hipGetLastError();
}

hipError_t ile_launch_hist_cdf(int nb, const double *P, double *C, hipStream_t st)
{
    hipLaunchKernelGGL(k_hist_cdf, dim3(1), dim3(64), 0, st, nb, P, C);
    return hipGetLastError();
}

hipError_t ile_launch_hist_draw(uint64_t seed, int64_t first, int64_t N, int nb,
                                const double *P, const double *C, double d_min,
                                double d_max, double t_ref_max, double *smp, int64_t ld,
                                double *ln_p, double *ln_q, int32_t *bins, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist_draw, dim3(nblk(N, 256)), dim3(256), 0, st, seed, first, N,
                       nb, P, C, d_min, d_max, t_ref_max, smp, ld, ln_p, ln_q, bins);
    return hipGetLastError();
}

size_t ile_hist_refit_tmp_doubles(int64_t N, int nb)
{
    const int64_t nblocks = std::min<int64_t>((N + 4095) / 4096, 4096);
    return 2 * kStatBlocks + 4 + (size_t)std::max<int64_t>(nblocks, 1) * 2 * nb;
}

hipError_t ile_launch_hist_refit(const int32_t *bins, int64_t ld, const double *lnL,
                                 const double *ln_p, const double *ln_q, int64_t N, int nb,
                                 double floor_w, double scale, double *tmp, double *P,
                                 double *C, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    double *part_stats = tmp, *stats = tmp + 2 * kStatBlocks, *part = stats + 4;
    hipLaunchKernelGGL(k_lnw_stats, dim3(kStatBlocks), dim3(kStatT), 0, st, lnL, ln_p,
                       ln_q, N, part_stats);
    hipLaunchKernelGGL(k_lnw_beta, dim3(1), dim3(64), 0, st, (const double *)part_stats,
                       N, scale, stats);
    const int64_t nblocks = std::min<int64_t>((N + 4095) / 4096, 4096);
    const int64_t per_block = (N + nblocks - 1) / nblocks;
    const size_t lds = (size_t)kHistT * 2 * nb * sizeof(double);
    hipLaunchKernelGGL(k_hist_partial, dim3((unsigned)nblocks), dim3(kHistT), lds, st, bins,
                       ld, lnL, ln_p, ln_q, N, nb, per_block, (const double *)stats, part);
    hipLaunchKernelGGL(k_hist_finish, dim3(1), dim3(256), 0, st, (const double *)part,
                       (int)nblocks, nb, floor_w, P, C);
    return hipGetLastError();
}
