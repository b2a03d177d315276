// Extrinsic posterior harvest (Sec. V: joint intrinsic and extrinsic
// information from one final Monte Carlo iteration; Eq. (3) at fixed
// intrinsic parameters).  The draws theta_alpha with log prior ln p and log
// proposal ln q and the bin grid t_j of Eq. (9) carry the joint weight
// exp(ln p - ln q + L_alpha,j); a draw takes the sample by inverse CDF of the
// Eq. (4) weights exp(lnLmargT + ln p - ln q), then the bin by inverse CDF of
// exp(L_alpha,j) for that sample.
//
//   k_hv_lw    ln w per sample and per-block maxima
//   k_hv_max   max ln w over the block maxima
//   k_hv_w     w = exp(ln w - max ln w)        (then the fixed-order prefix
//                                               sums of ile_launch_mdn_cdf)
//   k_hv_pick  sample index per draw (binary search of the cumulative sums;
//              u is [2][n_out], both rows are checked here)
//   k_hv_gather  the chosen samples, packed, for the per-bin evaluation
//   k_hv_bin   one wave per draw: the bin from the cumulative sums of
//              exp(L_j - max L), and the harvested parameters (k_hv_bin_seg
//              up to 2048 bins: row in registers, lane-owned segments in
//              LDS; above, k_hv_bin streams the row with chunked wave scans)
#include "ile_internal.h"

#include <math.h>

namespace {

constexpr int HV_T = 256;

__device__ inline double wave_max_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(HV_T) void k_hv_lw(const double *__restrict__ lnL,
                                                const double *__restrict__ lp,
                                                const double *__restrict__ lq, int64_t n,
                                                double *__restrict__ lw, double *__restrict__ part,
                                                int32_t *err)
{
    __shared__ double sm[HV_T / 64];
    double m = -INFINITY;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * HV_T + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * HV_T) {
        const double p = lp ? lp[i] : 0.0, q = lq ? lq[i] : 0.0;
        // ln p = -inf is a zero weight; NaN, ln p = +inf and ln q = -inf are
        // not densities
        bad |= isnan(p) || isnan(q) || p == INFINITY || q == -INFINITY;
        const double v = lnL[i] + p - q;
        const double x = isnan(v) ? -INFINITY : v;
        lw[i] = x;
        m = fmax(m, x);
    }
    if (bad) atomicOr(err, 1);
    m = wave_max_d(m);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sm[0];
        for (int w = 1; w < HV_T / 64; w++) b = fmax(b, sm[w]);
        part[blockIdx.x] = b;
    }
}

// max ln w over the per-block maxima into part[n_part] (one block)
__global__ __launch_bounds__(64) void k_hv_max(double *part, int n_part)
{
    double m = -INFINITY;
    for (int b = threadIdx.x; b < n_part; b += 64) m = fmax(m, part[b]);
    m = wave_max_d(m);
    if (threadIdx.x == 0) part[n_part] = m;
}

__global__ __launch_bounds__(HV_T) void k_hv_w(double *__restrict__ w, int64_t n,
                                               const double *__restrict__ pM, int32_t *err)
{
    const double M = *pM;
    const int64_t i = (int64_t)blockIdx.x * HV_T + threadIdx.x;
    if (M == -INFINITY || M == INFINITY) {
        if (i == 0) atomicOr(err, 2);   // no sample with a finite positive weight
        if (i < n) w[i] = 0.0;
        return;
    }
    if (i < n) w[i] = exp(w[i] - M);
}

// first index with cdf > target; if rounding leaves none, the first index
// whose cumulative weight reaches the total (never a zero-weight sample)
__device__ inline int64_t inverse_cdf(const double *__restrict__ cdf, int64_t n, double target)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    if (cdf[lo] > target) return lo;
    const double tot = cdf[n - 1];
    lo = 0;
    hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] >= tot)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(HV_T) void k_hv_pick(const double *__restrict__ cdf, int64_t n,
                                                  const double *__restrict__ u, int64_t n_out,
                                                  int64_t *__restrict__ idx, int32_t *err)
{
    const int64_t k = (int64_t)blockIdx.x * HV_T + threadIdx.x;
    if (k >= n_out) return;
    const double uk = u[k], vk = u[n_out + k];
    if (!(uk >= 0.0 && uk < 1.0 && vk >= 0.0 && vk < 1.0)) {
        atomicOr(err, 4);
        idx[k] = 0;
        return;
    }
    idx[k] = inverse_cdf(cdf, n, uk * cdf[n - 1]);
}

__global__ __launch_bounds__(HV_T) void k_hv_gather(const double *__restrict__ smp, int64_t ld,
                                                    const int64_t *__restrict__ idx, int64_t m,
                                                    double *__restrict__ sel)
{
    const int64_t r = (int64_t)blockIdx.x * HV_T + threadIdx.x;
    if (r >= m) return;
    const int64_t a = idx[r];
#pragma unroll
    for (int p = 0; p < 7; p++) sel[p * m + r] = smp[p * ld + a];
}

// Cumulative bin weights of one chunk of 64 bins: exp(L_j - M) summed in
// order within the wave (inclusive scan), offset by the running total of
// the earlier chunks.  Both passes over a row call this, so the values the
// search sees are exactly the ones that built the total.
__device__ inline double chunk_cdf(const double *__restrict__ L, int base, int n_t, double M,
                                   double run, int lane, double &chunk_tot)
{
    const int j = base + lane;
    double x = j < n_t ? exp(L[j] - M) : 0.0;
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    chunk_tot = __shfl(x, 63, 64);
    return run + x;
}

__global__ __launch_bounds__(HV_T) void k_hv_bin(const double *__restrict__ series, int64_t m,
                                                 int n_t, const double *__restrict__ v,
                                                 const double *__restrict__ sel, double srate,
                                                 int32_t *__restrict__ bins,
                                                 double *__restrict__ theta, int64_t ld_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (HV_T / 64) + (threadIdx.x >> 6);
    if (r >= m) return;   // whole waves leave together
    const double *L = series + r * n_t;
    double M = -INFINITY;
    for (int j = lane; j < n_t; j += 64) M = fmax(M, L[j]);
    M = wave_max_d(M);
    double run = 0.0, ct;
    for (int base = 0; base < n_t; base += 64) {
        chunk_cdf(L, base, n_t, M, run, lane, ct);
        run += ct;
    }
    const double tot = run, target = v[r] * tot;
    int jsel = -1;
    run = 0.0;
    for (int base = 0; base < n_t && jsel < 0; base += 64) {
        const double c = chunk_cdf(L, base, n_t, M, run, lane, ct);
        const uint64_t hit = __ballot(base + lane < n_t && c > target);
        if (hit) jsel = base + __builtin_ctzll(hit);
        run += ct;
    }
    run = 0.0;
    for (int base = 0; base < n_t && jsel < 0; base += 64) {
        const double c = chunk_cdf(L, base, n_t, M, run, lane, ct);
        const uint64_t hit = __ballot(base + lane < n_t && c >= tot);
        if (hit) jsel = base + __builtin_ctzll(hit);
        run += ct;
    }
    if (theta && lane < 7) {
        double x = sel[lane * m + r];
        if (lane == 6) x += (double)(jsel - (n_t - 1) / 2) / srate;
        theta[lane * ld_out + r] = x;
    }
    if (lane == 0) bins[r] = jsel;
}

// Segment form of the pick (n_t <= 64 NC): the row is read once into
// registers, its weights exp(L_j - M) go through the wave's own LDS region
// so that lane l owns the contiguous bins [l S, (l + 1) S), S = ceil(n_t /
// 64).  Each lane sums its segment in order (T_l); a wave scan gives the
// offsets E_l; the cumulative weight of bin j = l S + k is E_l + (sum of the
// segment's first k + 1 weights), which at a segment's end is E_l + T_l, and
// the total is that of the last lane.  The first lane whose segment end
// exceeds the target scans its segment for the bin (when rounding leaves no
// such lane, the first bin reaching the total).  Two dependent passes of S
// steps and one 6-step scan, where k_hv_bin chains a scan per 64-bin chunk.
__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NC>
__global__ __launch_bounds__(HV_T) void k_hv_bin_seg(const double *__restrict__ series, int64_t m,
                                                     int n_t, const double *__restrict__ v,
                                                     const double *__restrict__ sel, double srate,
                                                     int32_t *__restrict__ bins,
                                                     double *__restrict__ theta, int64_t ld_out)
{
    extern __shared__ double hv_seg[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * (HV_T / 64) + wv;
    if (r >= m) return;   // whole waves; each uses only its own LDS region
    const int S = (n_t + 63) >> 6;
    double *e = hv_seg + wv * 64 * S;
    const double *L = series + r * n_t;
    double x[NC];
    double M = -INFINITY;
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const int j = c * 64 + lane;
        x[c] = (c < S && j < n_t) ? L[j] : -INFINITY;
        M = fmax(M, x[c]);
    }
    M = wave_max_d(M);
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const int j = c * 64 + lane;
        if (c < S) e[j] = j < n_t ? exp(x[c] - M) : 0.0;
    }
    wave_sync_lds();
    const double *mine = e + lane * S;
    double T = 0.0;
    for (int k = 0; k < S; k++) T += mine[k];
    double P = T;   // inclusive scan over lanes
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(P, o, 64);
        if (lane >= o) P += y;
    }
    double E = __shfl_up(P, 1, 64);
    if (lane == 0) E = 0.0;
    const double end = E + T;
    const double tot = __shfl(end, 63, 64), target = v[r] * tot;
    uint64_t hit = __ballot(end > target);
    const bool reach = hit == 0;   // rounding left the target at the total
    if (reach) hit = __ballot(end >= tot);
    const int owner = __builtin_ctzll(hit);
    int jl = 0;
    if (lane == owner) {
        double q = 0.0;
        for (int k = 0; k < S; k++) {
            q += mine[k];
            const double cj = E + q;
            if (reach ? cj >= tot : cj > target) {
                jl = lane * S + k;
                break;
            }
        }
    }
    const int jsel = __shfl(jl, owner, 64);
    if (theta && lane < 7) {
        double y = sel[lane * m + r];
        if (lane == 6) y += (double)(jsel - (n_t - 1) / 2) / srate;
        theta[lane * ld_out + r] = y;
    }
    if (lane == 0) bins[r] = jsel;
}

}  // namespace

int ile_hv_parts() { return 256; }

hipError_t ile_launch_hv_weights(const double *lnL, const double *ln_p, const double *ln_q,
                                 int64_t n, double *w, double *part, int32_t *err,
                                 hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nb = ile_hv_parts();
    hipLaunchKernelGGL(k_hv_lw, dim3(nb), dim3(HV_T), 0, st, lnL, ln_p, ln_q, n, w, part, err);
    hipLaunchKernelGGL(k_hv_max, dim3(1), dim3(64), 0, st, part, nb);
    hipLaunchKernelGGL(k_hv_w, dim3((unsigned)((n + HV_T - 1) / HV_T)), dim3(HV_T), 0, st, w, n,
                       (const double *)(part + nb), err);
    return hipGetLastError();
}

hipError_t ile_launch_hv_pick(const double *cdf, int64_t n, const double *u, int64_t n_out,
                              int64_t *idx, int32_t *err, hipStream_t st)
{
    if (n_out <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hv_pick, dim3((unsigned)((n_out + HV_T - 1) / HV_T)), dim3(HV_T), 0, st,
                       cdf, n, u, n_out, idx, err);
    return hipGetLastError();
}

hipError_t ile_launch_hv_gather(const double *smp, int64_t ld, const int64_t *idx, int64_t m,
                                double *sel, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hv_gather, dim3((unsigned)((m + HV_T - 1) / HV_T)), dim3(HV_T), 0, st,
                       smp, ld, idx, m, sel);
    return hipGetLastError();
}

hipError_t ile_launch_hv_bin(const double *series, int64_t m, int n_t, const double *v,
                             const double *sel, double srate, int32_t *bins, double *theta,
                             int64_t ld_out, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    constexpr int rows = HV_T / 64;
    const dim3 grid((unsigned)((m + rows - 1) / rows));
    const size_t seg = (size_t)rows * 64 * ((n_t + 63) / 64) * sizeof(double);
    if (n_t <= 64 * 8)
        hipLaunchKernelGGL(k_hv_bin_seg<8>, grid, dim3(HV_T), seg, st, series, m, n_t, v, sel, srate,
                           bins, theta, ld_out);
    else if (n_t <= 64 * 32)
        hipLaunchKernelGGL(k_hv_bin_seg<32>, grid, dim3(HV_T), seg, st, series, m, n_t, v, sel,
                           srate, bins, theta, ld_out);
    else
        hipLaunchKernelGGL(k_hv_bin, grid, dim3(HV_T), 0, st, series, m, n_t, v, sel, srate, bins,
                           theta, ld_out);
    return hipGetLastError();
}
