// Q, U, V of Eq. (8) from frequency-domain series: the band-limited,
// noise-weighted inner products of Eq. (2) as sums over the n-point FFT grid
// f_i = i df (i < n/2), (i - n) df (i >= n/2).
//
//   k_fd_prod   X_k,lm,i = 2 df / S_k,i conj(h_lm,i) d_k,i exp(2 pi i f_i t0)
//               (0 outside f_min < |f_i| < f_max)
//   k_fft_row   inverse FFT of one row in LDS (n <= 1024), or for larger
//   k_fft_a/c   n = N1 N2 the four-step form: N1 transforms of length N2 over
//               strided columns, a twiddle, N2 transforms of length N1; each
//               transform self-sorting radix-2 passes in LDS:
//               Q_k,lm[s] = sum_i X_k,lm,i exp(2 pi i i s / n), Q at t0 + s / (n df)
//   k_uv        U_k[a][b] = sum_i w_k,i conj(h_a,i) h_b,i and
//               V_k[a][b] = sum_i w_k,i h_a,-i h_b,i (w = 2 df / S in the
//               band), one workgroup per (k, a, b), fixed-order reduction
#include "ile_internal.h"

#include <math.h>

#include <algorithm>

namespace {

constexpr int FD_T = 256;

__device__ inline double fd_freq(int64_t i, int64_t n, double df)
{
    return (double)(i < n / 2 ? i : i - n) * df;
}

// 2 df / S in the open band, else 0; bit 0 of err for a bad spectrum there
__device__ inline double fd_weight(double f, double S, double df, double f_min, double f_max,
                                   bool &bad)
{
    const double af = fabs(f);
    if (!(af > f_min && af < f_max)) return 0.0;
    if (!(S > 0.0) || !isfinite(S)) {
        bad = true;
        return 0.0;
    }
    return 2.0 * df / S;
}

__global__ __launch_bounds__(FD_T) void k_fd_prod(const double2 *__restrict__ h,
                                                  const double2 *__restrict__ d,
                                                  const double *__restrict__ psd, int64_t n,
                                                  int n_det, int n_lm, double df, double f_min,
                                                  double f_max, double t0,
                                                  double2 *__restrict__ X, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * FD_T + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n) return;
    const double f = fd_freq(i, n, df);
    bool bad = false;
    const double w = fd_weight(f, psd[(int64_t)k * n + i], df, f_min, f_max, bad);
    const double2 dk = d[(int64_t)k * n + i];
    bad |= !isfinite(dk.x) || !isfinite(dk.y);
    double sn, cs;
    sincospi(2.0 * f * t0, &sn, &cs);
    // g = w d exp(2 pi i f t0)
    const double gx = w * (dk.x * cs - dk.y * sn), gy = w * (dk.x * sn + dk.y * cs);
    for (int a = 0; a < n_lm; a++) {
        const double2 ha = h[(int64_t)a * n + i];
        bad |= !isfinite(ha.x) || !isfinite(ha.y);
        // conj(h) g
        X[((int64_t)k * n_lm + a) * n + i] =
            make_double2(ha.x * gx + ha.y * gy, ha.x * gy - ha.y * gx);
    }
    if (bad) atomicOr(err, 1);
}

// Inverse DFT (unnormalized, exp(+2 pi i jk/L)) of nb sequences of length L
// held at a + q L, by self-sorting radix-2 passes ping-ponging between a and
// b (pass with sub-length len, stride st = L / len: for t = p st + q',
// u = a[q' + st p], v = a[q' + st (p + len/2)], b[q' + 2 st p] = u + v,
// b[q' + st (2p + 1)] = (u - v) exp(2 pi i p / len)).  tw[j] = exp(2 pi i j / L)
// for j < L/2 (exp(2 pi i p / len) = tw[p st], the same value).  Returns the
// buffer holding the result.  Every thread of the block must call it.
__device__ inline void lds_twiddles(double2 *tw, int L)
{
    for (int j = threadIdx.x; j < L / 2; j += FD_T) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)L, &sn, &cs);
        tw[j] = make_double2(cs, sn);
    }
}

__device__ double2 *lds_ifft(double2 *a, double2 *b, const double2 *tw, int nb, int L)
{
    const int hl = L / 2, tot = nb * hl;
    for (int len = L, st = 1; len > 1; len >>= 1, st <<= 1) {
        for (int t = threadIdx.x; t < tot; t += FD_T) {
            const int sq = t / hl, w = t - sq * hl;
            const int p = w / st, q = w - p * st;
            const double2 *x = a + sq * L;
            double2 *y = b + sq * L;
            const double2 u = x[q + st * p], v = x[q + st * (p + len / 2)];
            const double cs = tw[p * st].x, sn = tw[p * st].y;
            const double dx = u.x - v.x, dy = u.y - v.y;
            y[q + st * 2 * p] = make_double2(u.x + v.x, u.y + v.y);
            y[q + st * (2 * p + 1)] = make_double2(dx * cs - dy * sn, dx * sn + dy * cs);
        }
        __syncthreads();
        double2 *tmp = a;
        a = b;
        b = tmp;
    }
    return a;
}

// one workgroup per row, the whole row in LDS (n <= 1024)
__global__ __launch_bounds__(FD_T) void k_fft_row(const double2 *__restrict__ x,
                                                  double2 *__restrict__ y, int n)
{
    extern __shared__ double2 sh[];
    const int64_t row = (int64_t)blockIdx.x * n;
    for (int e = threadIdx.x; e < n; e += FD_T) sh[e] = x[row + e];
    lds_twiddles(sh + 2 * n, n);
    __syncthreads();
    const double2 *r = lds_ifft(sh, sh + n, sh + 2 * n, 1, n);
    for (int e = threadIdx.x; e < n; e += FD_T) y[row + e] = r[e];
}

// Four-step, first half: columns i1 in [c0, c0 + B) of the N1 x N2 view
// x[i1 + N1 i2]; transform over i2, twiddle exp(2 pi i i1 s2 / n), store
// t[s2 N1 + i1] (B consecutive i1: contiguous).
__global__ __launch_bounds__(FD_T) void k_fft_a(const double2 *__restrict__ x,
                                                double2 *__restrict__ t, int64_t n, int N1,
                                                int N2, int B)
{
    extern __shared__ double2 sh[];
    const int64_t row = (int64_t)blockIdx.y * n;
    const int c0 = blockIdx.x * B;
    for (int e = threadIdx.x; e < B * N2; e += FD_T) {
        const int b = e % B, i2 = e / B;
        sh[b * N2 + i2] = x[row + c0 + b + (int64_t)N1 * i2];
    }
    lds_twiddles(sh + 2 * B * N2, N2);
    __syncthreads();
    const double2 *r = lds_ifft(sh, sh + B * N2, sh + 2 * B * N2, B, N2);
    for (int e = threadIdx.x; e < B * N2; e += FD_T) {
        const int b = e % B, s2 = e / B;
        const int64_t i1 = c0 + b;
        const double2 z = r[b * N2 + s2];
        double sn, cs;
        sincospi(2.0 * (double)((i1 * s2) % n) / (double)n, &sn, &cs);
        t[row + (int64_t)s2 * N1 + i1] = make_double2(z.x * cs - z.y * sn, z.x * sn + z.y * cs);
    }
}

// Four-step, second half: rows s2 in [d0, d0 + B) of t (contiguous over
// i1); transform over i1 and store y[s2 + N2 s1].
__global__ __launch_bounds__(FD_T) void k_fft_c(const double2 *__restrict__ t,
                                                double2 *__restrict__ y, int64_t n, int N1,
                                                int N2, int B)
{
    extern __shared__ double2 sh[];
    const int64_t row = (int64_t)blockIdx.y * n;
    const int d0 = blockIdx.x * B;
    for (int e = threadIdx.x; e < B * N1; e += FD_T) {
        const int i1 = e % N1, b = e / N1;
        sh[b * N1 + i1] = t[row + (int64_t)(d0 + b) * N1 + i1];
    }
    lds_twiddles(sh + 2 * B * N1, N1);
    __syncthreads();
    const double2 *r = lds_ifft(sh, sh + B * N1, sh + 2 * B * N1, B, N1);
    for (int e = threadIdx.x; e < B * N1; e += FD_T) {
        const int b = e % B, s1 = e / B;
        y[row + d0 + b + (int64_t)N2 * s1] = r[b * N1 + s1];
    }
}

__global__ __launch_bounds__(FD_T) void k_uv(const double2 *__restrict__ h,
                                             const double *__restrict__ psd, int64_t n, int n_lm,
                                             double df, double f_min, double f_max,
                                             double2 *__restrict__ U, double2 *__restrict__ V)
{
    __shared__ double red[4][FD_T];
    const int b = blockIdx.x, a = blockIdx.y, k = blockIdx.z;
    const double2 *ha = h + (int64_t)a * n, *hb = h + (int64_t)b * n;
    const double *S = psd + (int64_t)k * n;
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    bool bad = false;
    for (int64_t i = threadIdx.x; i < n; i += FD_T) {
        const double w = fd_weight(fd_freq(i, n, df), S[i], df, f_min, f_max, bad);
        if (w == 0.0) continue;
        const double2 x = ha[i], y = hb[i], z = ha[i == 0 ? 0 : n - i];
        ur += w * (x.x * y.x + x.y * y.y);   // conj(x) y
        ui += w * (x.x * y.y - x.y * y.x);
        vr += w * (z.x * y.x - z.y * y.y);   // z y
        vi += w * (z.x * y.y + z.y * y.x);
    }
    red[0][threadIdx.x] = ur;
    red[1][threadIdx.x] = ui;
    red[2][threadIdx.x] = vr;
    red[3][threadIdx.x] = vi;
    __syncthreads();
    for (int o = FD_T / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < 4; c++) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)k * n_lm + a) * n_lm + b;
        U[o] = make_double2(red[0][0], red[1][0]);
        V[o] = make_double2(red[2][0], red[3][0]);
    }
}

}  // namespace

hipError_t ile_launch_fd_prod(const double *h, const double *d, const double *psd, int64_t n,
                              int n_det, int n_lm, double df, double f_min, double f_max,
                              double t0, double *X, int32_t *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_fd_prod, dim3((unsigned)((n + FD_T - 1) / FD_T), n_det), dim3(FD_T), 0, st,
                       (const double2 *)h, (const double2 *)d, psd, n, n_det, n_lm, df, f_min,
                       f_max, t0, (double2 *)X, err);
    return hipGetLastError();
}

// 1024 complex doubles per transform batch: 2 x 16 KB of LDS (ping-pong)
// plus the twiddle table (at most 8 KB), within 64 KB per workgroup; the
// four-step form then reaches n = 1024^2 = 2^20
constexpr int FFT_LDS = 1024;

int ile_fft_passes(int64_t n)
{
    return n <= FFT_LDS ? 1 : 2;   // kernels, each reading one buffer and writing the other
}

hipError_t ile_launch_ifft_rows(double *a, double *b, int64_t n, int rows, double **result,
                                hipStream_t st)
{
    const double2 *x = (const double2 *)a;
    double2 *y = (double2 *)b;
    if (n <= FFT_LDS) {
        hipLaunchKernelGGL(k_fft_row, dim3(rows), dim3(FD_T), (2 * n + n / 2) * sizeof(double2), st,
                           x, y, (int)n);
        *result = b;
        return hipGetLastError();
    }
    int lg = 0;
    while (((int64_t)1 << lg) < n) lg++;
    const int N2 = 1 << (lg / 2), N1 = (int)(n / N2);   // both <= 1024 for n <= 2^20
    const int BA = std::min(16, FFT_LDS / N2), BC = std::min(16, FFT_LDS / N1);
    hipLaunchKernelGGL(k_fft_a, dim3(N1 / BA, rows), dim3(FD_T),
                       (2 * BA * N2 + N2 / 2) * sizeof(double2), st, x, y, n, N1, N2, BA);
    hipLaunchKernelGGL(k_fft_c, dim3(N2 / BC, rows), dim3(FD_T),
                       (2 * BC * N1 + N1 / 2) * sizeof(double2), st, (const double2 *)y, (double2 *)a,
                       n, N1, N2, BC);
    *result = a;
    return hipGetLastError();
}

hipError_t ile_launch_uv_fd(const double *h, const double *psd, int64_t n, int n_det, int n_lm,
                            double df, double f_min, double f_max, double *U, double *V,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_uv, dim3(n_lm, n_lm, n_det), dim3(FD_T), 0, st, (const double2 *)h, psd,
                       n, n_lm, df, f_min, f_max, (double2 *)U, (double2 *)V);
    return hipGetLastError();
}
