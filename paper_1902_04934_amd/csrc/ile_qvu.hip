// Q, U, V of Eq. (8) from frequency-domain series: the band-limited,
// noise-weighted inner products of Eq. (2) as sums over the n-point FFT grid
// f_i = i df (i < n/2), (i - n) df (i >= n/2).
//
//   k_fd_prod   X_k,lm,i = 2 df / S_k,i conj(h_lm,i) d_k,i exp(2 pi i f_i t0)
//               (0 outside f_min < |f_i| < f_max)
//   k_fft_pass4 one radix-4 pass of a self-sorting (Stockham) inverse FFT
//               over all n_det n_lm rows (k_fft_pass: one radix-2 pass
//               first when log2 n is odd): Q_k,lm[s] = sum_i X_k,lm,i
//               exp(2 pi i i s / n), i.e. Q at t0 + s / (n df)
//   k_uv        U_k[a][b] = sum_i w_k,i conj(h_a,i) h_b,i and
//               V_k[a][b] = sum_i w_k,i h_a,-i h_b,i (w = 2 df / S in the
//               band), one workgroup per (k, a, b), fixed-order reduction
#include "ile_internal.h"

#include <math.h>

#include <utility>

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

// Pass with current sub-transform length len and stride s = n / len: for
// t = p s + q (p < len/2, q < s), a = x[q + s p], b = x[q + s (p + len/2)],
// y[q + 2 s p] = a + b, y[q + s (2p + 1)] = (a - b) exp(2 pi i p / len).
__global__ __launch_bounds__(FD_T) void k_fft_pass(const double2 *__restrict__ x,
                                                   double2 *__restrict__ y, int64_t n,
                                                   int64_t len, int64_t s)
{
    const int64_t t = (int64_t)blockIdx.x * FD_T + threadIdx.x;
    if (t >= n / 2) return;
    const int64_t row = (int64_t)blockIdx.y * n;
    const int64_t p = t / s, q = t - p * s, half = len / 2;
    const double2 a = x[row + q + s * p], b = x[row + q + s * (p + half)];
    double sn, cs;
    sincospi(2.0 * (double)p / (double)len, &sn, &cs);
    const double dx = a.x - b.x, dy = a.y - b.y;
    y[row + q + s * 2 * p] = make_double2(a.x + b.x, a.y + b.y);
    y[row + q + s * (2 * p + 1)] = make_double2(dx * cs - dy * sn, dx * sn + dy * cs);
}

// Radix-4 pass, sub-transform length len, stride s = n / len: for
// t = p s + q (p < len/4), a_j = x[q + s (p + j len/4)], and with
// b0 = a0 + a2, b1 = a0 - a2, b2 = a1 + a3, b3 = i (a1 - a3), w = exp(2 pi i p / len):
// y[q + s 4p] = b0 + b2, y[q + s (4p+1)] = (b1 + b3) w,
// y[q + s (4p+2)] = (b0 - b2) w^2, y[q + s (4p+3)] = (b1 - b3) w^3.
__global__ __launch_bounds__(FD_T) void k_fft_pass4(const double2 *__restrict__ x,
                                                    double2 *__restrict__ y, int64_t n,
                                                    int64_t len, int64_t s)
{
    const int64_t t = (int64_t)blockIdx.x * FD_T + threadIdx.x;
    if (t >= n / 4) return;
    const int64_t row = (int64_t)blockIdx.y * n;
    const int64_t p = t / s, q = t - p * s, m = len / 4;
    const double2 a0 = x[row + q + s * p], a1 = x[row + q + s * (p + m)],
                  a2 = x[row + q + s * (p + 2 * m)], a3 = x[row + q + s * (p + 3 * m)];
    const double b0x = a0.x + a2.x, b0y = a0.y + a2.y, b1x = a0.x - a2.x, b1y = a0.y - a2.y;
    const double b2x = a1.x + a3.x, b2y = a1.y + a3.y;
    const double b3x = -(a1.y - a3.y), b3y = a1.x - a3.x;   // i (a1 - a3)
    const double fp = (double)p / (double)len;
    double s1, c1, s2, c2, s3, c3;
    sincospi(2.0 * fp, &s1, &c1);
    sincospi(4.0 * fp, &s2, &c2);
    sincospi(6.0 * fp, &s3, &c3);
    const double u1x = b1x + b3x, u1y = b1y + b3y, u2x = b0x - b2x, u2y = b0y - b2y;
    const double u3x = b1x - b3x, u3y = b1y - b3y;
    y[row + q + s * 4 * p] = make_double2(b0x + b2x, b0y + b2y);
    y[row + q + s * (4 * p + 1)] = make_double2(u1x * c1 - u1y * s1, u1x * s1 + u1y * c1);
    y[row + q + s * (4 * p + 2)] = make_double2(u2x * c2 - u2y * s2, u2x * s2 + u2y * c2);
    y[row + q + s * (4 * p + 3)] = make_double2(u3x * c3 - u3y * s3, u3x * s3 + u3y * c3);
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

int ile_fft_passes(int64_t n)
{
    int p = 0;
    while (((int64_t)1 << p) < n) p++;
    return (p & 1) + p / 2;   // one radix-2 pass if log2 n is odd, then radix-4
}

hipError_t ile_launch_ifft_rows(double *a, double *b, int64_t n, int rows, double **result,
                                hipStream_t st)
{
    double2 *x = (double2 *)a, *y = (double2 *)b;
    int64_t len = n, s = 1;
    int lg = 0;
    while (((int64_t)1 << lg) < n) lg++;
    if (lg & 1) {
        hipLaunchKernelGGL(k_fft_pass, dim3((unsigned)((n / 2 + FD_T - 1) / FD_T), rows),
                           dim3(FD_T), 0, st, (const double2 *)x, y, n, len, s);
        std::swap(x, y);
        len >>= 1;
        s <<= 1;
    }
    for (; len > 1; len >>= 2, s <<= 2) {
        hipLaunchKernelGGL(k_fft_pass4, dim3((unsigned)((n / 4 + FD_T - 1) / FD_T), rows),
                           dim3(FD_T), 0, st, (const double2 *)x, y, n, len, s);
        std::swap(x, y);
    }
    *result = (double *)x;
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
