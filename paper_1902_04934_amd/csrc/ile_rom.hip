// Surrogate (linear-basis) form (Sec. V): h_lm(lambda; t) = sum_b
// c_lm,b(lambda) e_b(t) with c_lm,b(lambda) = sum_p A[lm][b][p] lambda^p.
// Eq. (7) over the basis needs, per joint sample, the vector
//   z_b = sum_lm c_lm,b(lambda) -2Y_lm(iota, phi)
// in place of the harmonics; k_rom_z forms it (one thread per sample, the
// basis accumulators in registers) and the contraction reads it through
// ile_geom::ext_y.
#include "ile_internal.h"

#include <math.h>

namespace {

__global__ __launch_bounds__(256) void k_rom_z(const ile_geom gp, const double *__restrict__ smp,
                                               int64_t N, const double2 *__restrict__ A, int n_b,
                                               int n_pow, double2 *__restrict__ Z, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double lam = smp[7 * N + i], ci = smp[4 * N + i], phi = smp[3 * N + i];
    if (!(lam >= -1.0 && lam <= 1.0) || !(ci >= -1.0 && ci <= 1.0) || !isfinite(phi)) {
        atomicOr(err, 1);
        for (int b = 0; b < n_b; b++) Z[i * n_b + b] = make_double2(NAN, NAN);
        return;
    }
    double zx[ILE_MAX_LM], zy[ILE_MAX_LM];
#pragma unroll
    for (int b = 0; b < ILE_MAX_LM; b++) zx[b] = zy[b] = 0.0;
    for (int a = 0; a < gp.n_lm; a++) {
        const double2 y = sylm_dev(gp, a, ci, phi);
        const double2 *Aa = A + (int64_t)a * n_b * n_pow;
#pragma unroll
        for (int b = 0; b < ILE_MAX_LM; b++) {
            if (b < n_b) {
                const double2 *Ab = Aa + b * n_pow;
                double cx = Ab[n_pow - 1].x, cy = Ab[n_pow - 1].y;
                for (int p = n_pow - 2; p >= 0; p--) {   // Horner in lambda
                    cx = cx * lam + Ab[p].x;
                    cy = cy * lam + Ab[p].y;
                }
                zx[b] += cx * y.x - cy * y.y;
                zy[b] += cx * y.y + cy * y.x;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < ILE_MAX_LM; b++)
        if (b < n_b) Z[i * n_b + b] = make_double2(zx[b], zy[b]);
}

}  // namespace

hipError_t ile_launch_rom_z(const ile_geom &gp, const double *smp, int64_t N, const double *A,
                            int n_b, int n_pow, double *Z, int32_t *err, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rom_z, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, gp, smp, N,
                       (const double2 *)A, n_b, n_pow, (double2 *)Z, err);
    return hipGetLastError();
}
