// Surrogate (linear-basis) form (Sec. V): h_lm(lambda; t) = sum_b
// c_lm,b(lambda) e_b(t) with c_lm,b(lambda) = sum_p A[lm][b][p] lambda^p.
// Eq. (7) over the basis needs, per joint sample, the vector
//   z_b = sum_lm c_lm,b(lambda) -2Y_lm(iota, phi)
// in place of the harmonics; k_rom_z forms it (one thread per sample, the
// harmonics in registers) and the contraction reads it through
// ile_geom::ext_y.
#include "ile_internal.h"

#include <math.h>

namespace {

// A is staged in LDS when it fits (sA non-empty): every lane of a wave reads
// the same coefficient, an LDS broadcast instead of a scalar-cache miss.
__global__ __launch_bounds__(256) void k_rom_z(const ile_geom gp, const double *__restrict__ smp,
                                               int64_t N, const double2 *__restrict__ Ag, int n_b,
                                               int n_pow, int staged, double2 *__restrict__ Z,
                                               int32_t *err)
{
    extern __shared__ double2 sA[];
    const int nl = gp.n_lm;
    const int na = nl * n_b * n_pow;
    if (staged) {
        for (int e = threadIdx.x; e < na; e += 256) sA[e] = Ag[e];
        __syncthreads();
    }
    const double2 *A = staged ? sA : Ag;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double lam = smp[7 * N + i], ci = smp[4 * N + i], phi = smp[3 * N + i];
    if (!(lam >= -1.0 && lam <= 1.0) || !(ci >= -1.0 && ci <= 1.0) || !isfinite(phi)) {
        atomicOr(err, 1);
        for (int b = 0; b < n_b; b++) Z[i * n_b + b] = make_double2(NAN, NAN);
        return;
    }
    // the physical modes' harmonics in registers (unrolled, guarded)
    double yx[ILE_MAX_LM], yy[ILE_MAX_LM];
#pragma unroll
    for (int a = 0; a < ILE_MAX_LM; a++) {
        yx[a] = yy[a] = 0.0;
        if (a < nl) {
            const double2 y = sylm_dev(gp, a, ci, phi);
            yx[a] = y.x;
            yy[a] = y.y;
        }
    }
    for (int b = 0; b < n_b; b++) {
        double zx = 0.0, zy = 0.0;
#pragma unroll
        for (int a = 0; a < ILE_MAX_LM; a++) {
            if (a < nl) {
                const double2 *Ab = A + (a * n_b + b) * n_pow;
                double cx = Ab[n_pow - 1].x, cy = Ab[n_pow - 1].y;
                for (int p = n_pow - 2; p >= 0; p--) {   // Horner in lambda
                    cx = cx * lam + Ab[p].x;
                    cy = cy * lam + Ab[p].y;
                }
                zx += cx * yx[a] - cy * yy[a];
                zy += cx * yy[a] + cy * yx[a];
            }
        }
        Z[i * n_b + b] = make_double2(zx, zy);
    }
}

}  // namespace

hipError_t ile_launch_rom_z(const ile_geom &gp, const double *smp, int64_t N, const double *A,
                            int n_b, int n_pow, double *Z, int32_t *err, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    const size_t bytes = (size_t)gp.n_lm * n_b * n_pow * sizeof(double2);
    const int staged = bytes <= 64 * 1024;
    hipLaunchKernelGGL(k_rom_z, dim3((unsigned)((N + 255) / 256)), dim3(256), staged ? bytes : 0,
                       st, gp, smp, N, (const double2 *)A, n_b, n_pow, staged, (double2 *)Z, err);
    return hipGetLastError();
}
