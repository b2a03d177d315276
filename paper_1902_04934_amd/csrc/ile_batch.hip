// ile_batch.hip -- multi-point kernels of the batched form: many intrinsic
// points (uneven mode counts and window lengths) evaluated together
// (arXiv:1902.04934, Sec. III.B: each ILE instance loops over many
// intrinsic points to amortize its startup).  One launch each for the
// prior draw, window starts and ordering keys, scatter, and the per-point
// reduction; the contraction is the persistent kernel in ile_kernels.hip.
// Samples of point p live at offs[p] .. offs[p+1] of the concatenated
// arrays (SoA [7][N_p] per point); keys put point p in buckets
// [p B, (p+1) B) so one counting sort orders every point at once.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ile_internal.h"
#include "ile_rng.h"

namespace {

constexpr double kPi = 3.141592653589793238463;

__device__ inline int point_of(const int64_t *offs, int n_points, int64_t i)
{
    int lo = 0, hi = n_points - 1;   // last p with offs[p] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

using ile_rng::u53;

// prior draw: point p uses the Philox stream of key seed + p (the stream of
// ile_draw_prior_dev), sample t of the point counter t
__global__ __launch_bounds__(256) void k_prior_multi(const uint64_t *seed_dev,
                                                     const int64_t *offs, int n_points,
                                                     int64_t n_total, double d_min,
                                                     double d_max, double t_ref_max,
                                                     double *smp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int p = point_of(offs, n_points, i);
    const int64_t o = offs[p], n = offs[p + 1] - o, t = i - o;
    const uint64_t seed = *seed_dev + (uint64_t)p;
    uint32_t w[16];
    ile_rng::prior_words(seed, (uint64_t)t, w);
    double *s = smp + 7 * o;
    {
#pragma clang fp contract(off)
        const double v3 = d_max * d_max * d_max - d_min * d_min * d_min;
        s[0 * n + t] = 2.0 * kPi * u53(w[0], w[1]);
        s[1 * n + t] = asin(2.0 * u53(w[2], w[3]) - 1.0);
        s[2 * n + t] = kPi * u53(w[4], w[5]);
        s[3 * n + t] = 2.0 * kPi * u53(w[6], w[7]);
        s[4 * n + t] = 2.0 * u53(w[8], w[9]) - 1.0;
        s[5 * n + t] = cbrt(d_min * d_min * d_min + u53(w[10], w[11]) * v3);
        s[6 * n + t] = t_ref_max * (2.0 * u53(w[12], w[13]) - 1.0);
    }
}

// window starts and ordering keys (same arithmetic as the single-point path)
__global__ __launch_bounds__(256) void k_prep_multi(const ile_geom *geoms,
                                                    const int64_t *offs, int n_points,
                                                    int64_t n_total, const double *smp,
                                                    int32_t *shifts, uint32_t *keys,
                                                    uint32_t *hist, uint32_t B, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int p = point_of(offs, n_points, i);
    const ile_geom &g = geoms[p];
    const int64_t o = offs[p], n = offs[p + 1] - o, t = i - o;
    const double *s = smp + 7 * o;
    double th[7];
#pragma unroll
    for (int q = 0; q < 7; q++) th[q] = s[q * n + t];
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 7; q++) ok = ok && isfinite(th[q]);
    ok = ok && th[5] > 0.0 && th[4] >= -1.0 && th[4] <= 1.0 && fabs(th[6]) <= g.t_ref_max;
    int sh[ILE_MAX_DET];
    for (int k = 0; k < g.n_det; k++) {
        sh[k] = 0;
        if (ok) {
            double tau;
            {
#pragma clang fp contract(off)
                const double h = th[0] - g.gmst;
                const double n0 = cos(th[1]) * cos(h), n1 = cos(th[1]) * sin(h), n2 = sin(th[1]);
                const double nr = n0 * g.r[k][0] + n1 * g.r[k][1] + n2 * g.r[k][2];
                tau = -nr / 299792458.0;
            }
            double x;
            {
#pragma clang fp contract(off)
                x = (th[6] + tau - g.t0) / g.dt;
            }
            const double xs = floor(x + 0.5) - (double)g.half;
            if (xs >= 0.0 && xs <= (double)g.s_max)
                sh[k] = (int)xs;
            else
                ok = false;
        }
    }
    uint32_t key = B - 1;   // invalid samples last within the point
    if (ok) {
        key = cell_key(g, sh);
    } else {
        atomicOr(err, 1);
    }
    int32_t *shp = shifts + (int64_t)ILE_MAX_DET * o;
    for (int k = 0; k < g.n_det; k++) shp[(int64_t)k * n + t] = ok ? sh[k] : -1;
    key += (uint32_t)p * B;
    keys[i] = key;
    (void)wave_count_slot(hist, key);
}

// sorted position -> local sample index of the point
__global__ __launch_bounds__(256) void k_scatter_multi(const uint32_t *keys, const int64_t *offs,
                                                       int n_points, int64_t n_total,
                                                       uint32_t *pos, int32_t *perm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int p = point_of(offs, n_points, i);
    const uint32_t at = wave_count_slot(pos, keys[i]);
    perm[at] = (int32_t)(i - offs[p]);
}

// per-point importance-sampling partials (prior proposal: w = L), one
// workgroup per point, fixed-order tree: results[p] = {ln L_marg, n_eff,
// Kish, sigma, max lnLmargT, n}
constexpr int kRT = 1024;
// Per-point reduction: ln w = lnLmargT + (ln p - ln q) (lw = NULL: ln w =
// lnLmargT, the prior draws), fixed-order block sums; res[6 p ..] =
// (ln L_marg, n_eff, Kish, sigma, max lnLmargT, n).
__global__ __launch_bounds__(kRT) void k_reduce_points(const double *out, const double *lw,
                                                       const int64_t *offs, double *res)
{
    __shared__ double a[kRT], b[kRT];
    const int p = blockIdx.x, t = threadIdx.x;
    const int64_t o = offs[p], n = offs[p + 1] - o;
    double M = -INFINITY, ML = -INFINITY;
    for (int64_t i = t; i < n; i += kRT) {
        const double x = lw ? out[o + i] + lw[o + i] : out[o + i];
        M = fmax(M, x);
        ML = fmax(ML, out[o + i]);
    }
    a[t] = M;
    b[t] = ML;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
        if (t < s) {
            a[t] = fmax(a[t], a[t + s]);
            b[t] = fmax(b[t], b[t + s]);
        }
        __syncthreads();
    }
    M = a[0];
    ML = b[0];
    __syncthreads();
    double s1 = 0.0, s2 = 0.0;
    if (M != -INFINITY)
        for (int64_t i = t; i < n; i += kRT) {
            const double x = lw ? out[o + i] + lw[o + i] : out[o + i];
            const double e = exp(x - M);
            s1 += e;
            s2 += e * e;
        }
    a[t] = s1;
    b[t] = s2;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
        if (t < s) {
            a[t] += a[t + s];
            b[t] += b[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *r = res + 6 * p;
        if (M == -INFINITY || n == 0) {
            r[0] = -INFINITY;
            r[1] = r[2] = 0.0;
            r[3] = NAN;
        } else {
            r[0] = M + log(a[0]) - log((double)n);
            r[1] = a[0];
            r[2] = a[0] * a[0] / b[0];
            const double var = b[0] / (a[0] * a[0]) - 1.0 / (double)n;
            r[3] = var > 0.0 ? sqrt(var) : 0.0;
        }
        r[4] = ML;
        r[5] = (double)n;
    }
}

// ln p - ln q of caller-supplied draws (either may be NULL = 0); an invalid
// pair (NaN, ln q = -inf or ln p = +inf) sets bit 2 of the error flag.
__global__ __launch_bounds__(256) void k_batch_lw(const double *lp, const double *lq,
                                                  int64_t n_total, double *lw, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const double p = lp ? lp[i] : 0.0, q = lq ? lq[i] : 0.0;
    if (isnan(p) || isnan(q) || q == -INFINITY || p == INFINITY) {
        atomicOr(err, 2);
        lw[i] = NAN;
        return;
    }
    lw[i] = p - q;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t ile_launch_prior_multi(const uint64_t *seed_dev, const int64_t *offs, int n_points,
                                  int64_t n_total, double d_min, double d_max,
                                  double t_ref_max, double *smp, hipStream_t st)
{
    hipLaunchKernelGGL(k_prior_multi, dim3(nblk(n_total, 256)), dim3(256), 0, st, seed_dev,
                       offs, n_points, n_total, d_min, d_max, t_ref_max, smp);
    return hipGetLastError();
}

hipError_t ile_launch_prep_multi(const ile_geom *geoms, const int64_t *offs, int n_points,
                                 int64_t n_total, const double *smp, int32_t *shifts,
                                 uint32_t *keys, uint32_t *hist, uint32_t B, int32_t *err,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_prep_multi, dim3(nblk(n_total, 256)), dim3(256), 0, st, geoms, offs,
                       n_points, n_total, smp, shifts, keys, hist, B, err);
    return hipGetLastError();
}

hipError_t ile_launch_scatter_multi(const uint32_t *keys, const int64_t *offs, int n_points,
                                    int64_t n_total, uint32_t *pos, int32_t *perm,
                                    hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter_multi, dim3(nblk(n_total, 256)), dim3(256), 0, st, keys, offs,
                       n_points, n_total, pos, perm);
    return hipGetLastError();
}

hipError_t ile_launch_reduce_points(const double *out, const double *lw, const int64_t *offs,
                                    int n_points, double *res, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_points, dim3(n_points), dim3(kRT), 0, st, out, lw, offs, res);
    return hipGetLastError();
}

hipError_t ile_launch_batch_lw(const double *lp, const double *lq, int64_t n_total, double *lw,
                               int32_t *err, hipStream_t st)
{
    if (n_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_lw, dim3(nblk(n_total, 256)), dim3(256), 0, st, lp, lq, n_total,
                       lw, err);
    return hipGetLastError();
}
