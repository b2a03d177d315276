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

namespace {

constexpr double kPi = 3.141592653589793238463;
constexpr double kTwoPi = 6.283185307179586476925;

__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ inline double u53(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6) + 0.5) /
           9007199254740992.0;
}

// last bin b with C[b] <= u, and the position inside it
__device__ inline int invert(const double *P, const double *C, int nb, double u,
                             double &frac)
{
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid] <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    const double f = (u - C[lo]) / P[lo];
    frac = f < 1.0 ? f : 1.0;
    return lo;
}

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
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), b, 0x494C4531u};
        philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        w[4 * b] = c[0];
        w[4 * b + 1] = c[1];
        w[4 * b + 2] = c[2];
        w[4 * b + 3] = c[3];
    }
    double fr, fs;
    const int br = invert(sP, sC, nb, u53(w[0], w[1]), fr);
    const int bs = invert(sP + nb, sC + nb + 1, nb, u53(w[2], w[3]), fs);
    {
#pragma clang fp contract(off)
        const double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
        const double ra = ((double)br + fr) * (2.0 * kPi / nb);
        const double sd = -1.0 + ((double)bs + fs) * (2.0 / nb);
        const double dec = asin(sd);
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
        const double lp = -log(kTwoPi) + log(cos(dec) / 2.0) - log(kPi) - log(kTwoPi) -
                          log(2.0) + log(3.0 * D * D / v3) - log(2.0 * t_ref_max);
        if (ln_p) ln_p[t] = lp;
        if (ln_q) ln_q[t] = lp + log(nb * sP[br]) + log(nb * sP[nb + bs]);
    }
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
