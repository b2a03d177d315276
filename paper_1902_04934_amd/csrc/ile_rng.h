// ile_rng.h -- device random streams and draw mappings shared by the
// samplers.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): a counter-based generator, so draw i of a
// stream needs no state and every kernel can produce any sample's numbers
// on its own.  Counters are (i_lo, i_hi, block, stream tag) with the key =
// the run's seed; u53 turns two 32-bit words into a uniform in (0, 1) with
// 53 random bits.
#ifndef ILE_RNG_H
#define ILE_RNG_H
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ile_rng {

// stream tags (the fourth counter word)
constexpr uint32_t kTagPrior = 0x494C4531u;   // prior and histogram draws
constexpr uint32_t kTagMdn = 0x4D444E31u;     // learned-proposal draws
constexpr uint32_t kTagTrain = 0x4D444E54u;   // training minibatches

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
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

// one Philox block of stream `tag`, counter (i, block), key seed
__device__ inline void block(uint64_t seed, uint64_t i, uint32_t blk, uint32_t tag,
                             uint32_t out[4])
{
    out[0] = (uint32_t)i;
    out[1] = (uint32_t)(i >> 32);
    out[2] = blk;
    out[3] = tag;
    philox4x32_10(out, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline double u53(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6) + 0.5) /
           9007199254740992.0;
}

// the 16 words of the prior / histogram draw of sample i (blocks 0..3)
__device__ inline void prior_words(uint64_t seed, uint64_t i, uint32_t w[16])
{
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) block(seed, i, b, kTagPrior, &w[4 * b]);
}

// Prior density of a sample in the coordinates (ra, dec, psi, phi,
// cos iota, D, t_ref): uniform ra, psi, phi, cos iota and t_ref, p(dec) =
// cos(dec)/2, p(D) = 3 D^2 / (d_max^3 - d_min^3).
__device__ inline double ln_prior(double dec, double D, double d_min, double d_max,
                                  double t_ref_max)
{
#pragma clang fp contract(off)
    const double kPi_ = 3.141592653589793238463, kTwoPi_ = 6.283185307179586476925;
    const double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
    return -log(kTwoPi_) + log(cos(dec) / 2.0) - log(kPi_) - log(kTwoPi_) - log(2.0) +
           log(3.0 * D * D / v3) - log(2.0 * t_ref_max);
}

// last bin b of an nb-bin histogram (P, cumulative C) with C[b] <= u, and
// the position inside it
__device__ inline int hist_invert(const double *P, const double *C, int nb, double u,
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

// Draw of the histogram proposal from the 16 words of prior_words: ra and
// sin(dec) through the inverse CDFs of P[0..nb) and P[nb..2nb), the other
// parameters from the prior.  Returns ln p; x[7] receives the sample.
__device__ inline double hist_sample(const double *P, const double *C, int nb,
                                     const uint32_t w[16], double d_min, double d_max,
                                     double t_ref_max, double x[7], int &br, int &bs)
{
#pragma clang fp contract(off)
    double fr, fs;
    br = hist_invert(P, C, nb, u53(w[0], w[1]), fr);
    bs = hist_invert(P + nb, C + nb + 1, nb, u53(w[2], w[3]), fs);
    const double kPi_ = 3.141592653589793238463;
    const double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
    x[0] = ((double)br + fr) * (2.0 * kPi_ / nb);
    const double sd = -1.0 + ((double)bs + fs) * (2.0 / nb);
    x[1] = asin(sd);
    x[2] = kPi_ * u53(w[4], w[5]);
    x[3] = 2.0 * kPi_ * u53(w[6], w[7]);
    x[4] = 2.0 * u53(w[8], w[9]) - 1.0;
    x[5] = cbrt(d_min * d_min * d_min + u53(w[10], w[11]) * v3);
    x[6] = t_ref_max * (2.0 * u53(w[12], w[13]) - 1.0);
    return ln_prior(x[1], x[5], d_min, d_max, t_ref_max);
}

}  // namespace ile_rng
#endif
