// ile_internal.h -- device-side parameter blocks and launch wrappers shared
// by the HIP kernels (ile_kernels.hip) and the C-ABI host code (ile_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "ile.h"

// Enum fields and arguments arrive from C callers, where any int may sit in
// them; C++ must not load an out-of-range value as the enum type, so the
// ABI reads them as 32-bit integers and validates those.
template <typename E> inline int32_t enum_raw(const E &e)
{
    static_assert(sizeof(E) == sizeof(int32_t), "4-byte enum");
    int32_t v;
    memcpy(&v, &e, sizeof v);
    return v;
}

#define ILE_NPAR 7
#define ILE_MAX_TERMS 160   // Wigner-d terms over all modes (l <= 6, <= 32 modes)
#define ILE_LMAX 6

// Everything the kernels need about one intrinsic point and the detector
// network, passed by value as a kernel argument.
struct ile_geom {
    int n_det, n_lm, n_t, half;      // half = (n_t - 1) / 2
    int n_q;                         // length of each Q series
    int s_max;                       // largest valid window start, n_q - n_t
    // phased matrix-core engine: positions of one detector's G block (the
    // union of a chunk's windows) and the LDS row stride of that block; set
    // per launch from the LDS budget
    int wcap, wrow;
    double t0;                       // time of Q[0]
    double dt;                       // 1 / srate
    double d_ref, gmst, t_ref_max;
    double r[ILE_MAX_DET][3];        // site vectors [m]
    double D[ILE_MAX_DET][9];        // detector tensors
    // ordering key: Hilbert index of the window starts of up to 3 detectors
    int key_lo[3];
    int key_shift;                   // log2 of the cell width in samples
    int key_bits;                    // bits per axis
    int key_dims;                    // detectors used in the key
    // -2Y_lm as sums of a_t cos(i/2)^pc_t sin(i/2)^ps_t, times e^{i m phi}
    int mode_m[ILE_MAX_LM];
    int mode_first[ILE_MAX_LM];
    int mode_nterm[ILE_MAX_LM];
    double term_a[ILE_MAX_TERMS];
    // the powers pc_t | ps_t << 8, 32-bit so that the kernels read them with
    // scalar loads (a byte field of a kernel argument is a vector load)
    int term_pw[ILE_MAX_TERMS];
    int n_pw;                        // powers 0 .. n_pw - 1 of cos and sin(i/2) used
    int m_max;                       // largest |m| of the modes
    // surrogate form: per-sample vectors z [N][n_lm] used in place of -2Y_lm
    // (the n_lm "modes" are then basis functions), or null
    const double2 *ext_y;
};

// Device pointers of one intrinsic point of a batch.
struct ile_point_dev {
    const void *Q;            // planar Q (context precision)
    const double2 *U, *V;
    const double *smp;        // samples [7][N]
    int64_t N;
    const int32_t *perm;      // sorted order (local indices)
    const int32_t *shifts;    // window starts [n_det][N]
    double *out;              // lnLmargT [N]
    // phased engine: the point's per-sample terms (ile_launch_terms, tile
    // order from position 0), or null to form them in the tiles
    const double *terms;
};

// Increment table[key] by one for every active lane, aggregated over the
// lanes of the wave that share a key: one atomic per distinct key (the
// ordering keys of concentrated draws fall into few buckets, where one
// atomic per lane serializes).  Returns the lane's slot: the table value
// before the wave's increment plus the lane's rank among the lanes with its
// key.  The groups of equal keys are found first (register work only), then
// the first lane of every group issues its atomic, all of them in one
// instruction, so a wave waits for one atomic round trip however many
// distinct keys it holds.  Every active lane of the wave must call it.
__device__ inline uint32_t wave_count_slot(uint32_t *table, uint32_t key)
{
    uint64_t todo = __ballot(1);
    const int lane = __lane_id();
    int lead = lane;
    uint32_t rank = 0, cnt = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t k0 = __shfl(key, leader);
        const uint64_t same = __ballot(key == k0);
        if (key == k0) {
            lead = leader;
            rank = (uint32_t)__popcll(same & ((1ull << lane) - 1));
            cnt = (uint32_t)__popcll(same);
        }
        todo &= ~same;
    }
    uint32_t base = 0;
    if (lead == lane) base = atomicAdd(&table[key], cnt);
    return __shfl(base, lead) + rank;
}

// Ordering key of a sample: its cell (window starts of up to three
// detectors, each in cells of 2^key_shift positions, key_bits bits per axis)
// numbered along the Hilbert curve, so that runs of consecutive keys stay
// compact in every axis (tiles of consecutive samples then span narrower
// windows than along a Morton order).  Skilling's transpose form (J.
// Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 381, 2004),
// then the transposed bits interleaved from the most significant.
__device__ inline uint32_t cell_key(const ile_geom &g, const int *s)
{
    const int n = g.key_dims, b = g.key_bits;
    if (n < 1 || b < 1) return 0;   // a single cell
    uint32_t x[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (d < n) {
            int c = (s[d] - g.key_lo[d]) >> g.key_shift;
            c = c < 0 ? 0 : c;
            c = c > (1 << b) - 1 ? (1 << b) - 1 : c;
            x[d] = (uint32_t)c;
        }
    const uint32_t top = 1u << (b - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t p = q - 1;
#pragma unroll
        for (int i = 0; i < 3; i++)
            if (i < n) {
                if (x[i] & q) {
                    x[0] ^= p;
                } else {
                    const uint32_t t = (x[0] ^ x[i]) & p;
                    x[0] ^= t;
                    x[i] ^= t;
                }
            }
    }
#pragma unroll
    for (int i = 1; i < 3; i++)
        if (i < n) x[i] ^= x[i - 1];
    const uint32_t last = n == 3 ? x[2] : n == 2 ? x[1] : x[0];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (last & q) t ^= q - 1;
    uint32_t key = 0;
    for (int bit = b - 1; bit >= 0; bit--)
#pragma unroll
        for (int i = 0; i < 3; i++)
            if (i < n) key = (key << 1) | (((x[i] ^ t) >> bit) & 1u);
    return key;
}

// K steps of the matrix-core contraction (4 real rows = 2 modes each); the
// device Q holds 4 * ksp_of(n_lm) rows per detector (rows 2a and 2a+1 = Re,
// Im of mode a, the rest zero).
__device__ inline double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; i++) r *= x;
    return r;
}

// -2Y_lm(iota, phi) of mode a from the per-mode Wigner-d term table.
__device__ inline double2 sylm_dev(const ile_geom &g, int a, double cos_iota,
                                   double phi)
{
    double c = sqrt(0.5 * (1.0 + cos_iota));   // cos(iota/2)
    double s = sqrt(0.5 * (1.0 - cos_iota));   // sin(iota/2)
    double sum = 0.0;
    const int t0 = g.mode_first[a], nt = g.mode_nterm[a];
    for (int t = t0; t < t0 + nt; t++)
        sum += g.term_a[t] * ipow(c, g.term_pw[t] & 255) * ipow(s, g.term_pw[t] >> 8);
    double sm, cm;
    sincos((double)g.mode_m[a] * phi, &sm, &cm);
    return make_double2(sum * cm, sum * sm);
}

__host__ __device__ inline int ksp_of(int n_lm) { return (2 * n_lm + 3) / 4; }

// K steps (32 rows each) of the BF16 hi/lo contraction: the rows are
// [Q_hi (2 n_lm); Q_lo (2 n_lm); Q_hi (2 n_lm)], zero-padded; the device Q
// holds them K-contiguous per position: [n_det][n_q][32 * ksb_of(n_lm)] bf16.
__host__ __device__ inline int ksb_of(int n_lm) { return (6 * n_lm + 31) / 32; }

// Tuning of the contraction kernel.
struct ile_tune {
    int tile_samples;   // samples per workgroup tile (16)
    int threads;        // positions per G block of the pipelined engines: 128 .. 512
    int engine;         // 0: FMA on the vector ALUs, 1: matrix cores, producer and
                        // consumer waves; 3: matrix cores, phased waves
    int lds_budget;     // phased engine: dynamic LDS per workgroup in bytes (0: default)
};
bool ile_tune_supported(ile_precision prec, const ile_tune &tu);
// Sets the phased engine's block width in g (wcap, wrow) for this tuning;
// zero for the other engines.
void ile_contract_prepare(ile_geom &g, ile_precision prec, const ile_tune &tu);

// Launch wrappers (ile_kernels.hip).  All are asynchronous on `st`.
hipError_t ile_launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
hipError_t ile_launch_prep(const ile_geom &g, const double *smp, int64_t N,
                           int32_t *shifts, uint32_t *keys, uint32_t *hist,
                           uint32_t n_buckets, int32_t *err, hipStream_t st);
hipError_t ile_launch_scan(uint32_t *v, int64_t n, uint32_t *tmp, hipStream_t st);
int64_t ile_scan_tmp_words(int64_t n);
hipError_t ile_launch_scatter(const uint32_t *keys, int64_t N, uint32_t *offs,
                              int32_t *perm, hipStream_t st);
// The scatter plus copies of the samples [7][N] and window starts [nd][N]
// in tile order into smp_s, sh_s.
hipError_t ile_launch_scatter_copy(const uint32_t *keys, int64_t N, uint32_t *offs,
                                   int32_t *perm, const double *smp, const int32_t *shifts,
                                   int nd, double *smp_s, int32_t *sh_s, hipStream_t st);
hipError_t ile_launch_identity(int32_t *perm, int64_t N, hipStream_t st);
// Per-sample terms of Eq. (7) that the phased engine reads instead of
// forming them in its tiles (kernel k_terms, run by ile_launch_contract
// before the tiles that read them): for tile position i (sample perm[i])
// the fields f = 0 .. F - 1 (F = ile_terms_fields) at terms[16 F (r / 16) +
// 16 f + r % 16], r = i - t0, t0 the first position of the launch (a
// tile's fields are contiguous): q (the quadratic term), a validity flag (1
// or 0), (d_ref/D) F_k (re, im) for each detector, -2Y_lm (re, im) for
// each mode, then the window start of each detector; q, the F_k and the
// window starts are zero for an invalid sample.
int ile_terms_fields(const ile_geom &g);
bool ile_contract_uses_terms(ile_precision prec, const ile_tune &tu);
// The terms of positions 0 .. N-1 of one point into terms (16 F round16(N)
// doubles); uvt as for ile_launch_contract.
hipError_t ile_launch_terms(const ile_geom &g, const double *smp, int64_t N,
                            const int32_t *perm, const int32_t *shifts, const double *uvt,
                            double *terms, hipStream_t st);
// Positions per launch of the terms (a multiple of 16): the buffer for N
// samples holds ile_terms_fields x min(N, ILE_TERMS_CHUNK) doubles.
#define ILE_TERMS_CHUNK ((int64_t)1 << 21)
// uvt: per detector the upper triangles of the Hermitian part of U and the
// symmetric part of V, row by row, entry (a, b >= a) at 4 (a n_lm -
// a (a - 1) / 2 + b - a) as (Re U_h, Im U_h, Re V_s, Im V_s); terms: a buffer
// of ile_terms_fields x cap doubles, cap >= 16 a multiple of 16 (both used
// when ile_contract_uses_terms, else may be null).
// smp_s, sh_s: the samples and window starts already in tile order (the
// terms pass then reads them in order), or null (it gathers them through
// perm).
hipError_t ile_launch_contract(const ile_geom &g, ile_precision prec,
                               const ile_tune &tu, const double *smp, int64_t N,
                               const int32_t *perm, const int32_t *shifts,
                               const void *Q, const double *U, const double *V,
                               const double *smp_s, const int32_t *sh_s, const double *uvt,
                               double *terms, int64_t cap, double *out, double *series,
                               hipStream_t st);
size_t ile_contract_lds_bytes(const ile_geom &g, ile_precision prec,
                              const ile_tune &tu);
hipError_t ile_launch_prior(uint64_t seed, int64_t first, int64_t N,
                            double d_min, double d_max, double t_ref_max,
                            double *smp, int64_t ld, double *ln_p, hipStream_t st);
// Importance-sampling reduction of N values into a 5-double partial
// {M, S1, S2, n, maxL} with S1 = sum e^{lnw-M}, S2 = sum e^{2(lnw-M)}.
int ile_reduce_blocks();
hipError_t ile_launch_reduce(const double *lnL, const double *ln_p,
                             const double *ln_q, int64_t N, double *tmp,
                             double *partial, hipStream_t st);
// Merge n_part partials (fixed order) and finish into result[6].
hipError_t ile_launch_finish(const double *partials, int n_part, double *result,
                             hipStream_t st);
// Adaptive sampler (ile_sampler.hip): histogram state P[2][nb], C[2][nb+1].
int ile_hist_max_bins();
hipError_t ile_launch_hist_uniform(int nb, double *P, double *C, hipStream_t st);
hipError_t ile_launch_hist_cdf(int nb, const double *P, double *C, hipStream_t st);
hipError_t ile_launch_hist_draw(uint64_t seed, int64_t first, int64_t N, int nb,
                                const double *P, const double *C, double d_min,
                                double d_max, double t_ref_max, double *smp, int64_t ld,
                                double *ln_p, double *ln_q, int32_t *bins, hipStream_t st);
size_t ile_hist_refit_tmp_doubles(int64_t N, int nb);
hipError_t ile_launch_hist_refit(const int32_t *bins, int64_t ld, const double *lnL,
                                 const double *ln_p, const double *ln_q, int64_t N, int nb,
                                 double floor_w, double scale, double *tmp, double *P,
                                 double *C, hipStream_t st);
// Batched form (ile_batch.hip + the persistent contraction).
size_t ile_contract_dyn_bytes(const ile_geom &g, ile_precision prec, const ile_tune &tu);
// Allows the persistent kernel of this tuning `dyn` bytes of dynamic LDS;
// call outside stream capture, before ile_launch_contract_batched.
hipError_t ile_contract_batched_allow(ile_precision prec, const ile_tune &tu, size_t dyn);
hipError_t ile_launch_contract_batched(ile_precision prec, const ile_tune &tu,
                                       const ile_geom *geoms, const ile_point_dev *pts,
                                       const int2 *items, int n_items, unsigned *counter,
                                       int grid, size_t dyn, bool terms, hipStream_t st);
hipError_t ile_launch_prior_multi(const uint64_t *seed_dev, const int64_t *offs, int n_points,
                                  int64_t n_total, double d_min, double d_max,
                                  double t_ref_max, double *smp, hipStream_t st);
hipError_t ile_launch_prep_multi(const ile_geom *geoms, const int64_t *offs, int n_points,
                                 int64_t n_total, const double *smp, int32_t *shifts,
                                 uint32_t *keys, uint32_t *hist, uint32_t B, int32_t *err,
                                 hipStream_t st);
hipError_t ile_launch_scatter_multi(const uint32_t *keys, const int64_t *offs, int n_points,
                                    int64_t n_total, uint32_t *pos, int32_t *perm,
                                    hipStream_t st);
hipError_t ile_launch_reduce_points(const double *out, const double *lw, const int64_t *offs,
                                    int n_points, double *res, hipStream_t st);
hipError_t ile_launch_batch_lw(const double *lp, const double *lq, int64_t n_total, double *lw,
                               int32_t *err, hipStream_t st);
hipError_t ile_launch_to_bf16_split(const double *Q, int64_t n, void *dst,
                                    hipStream_t st);

// ------------------------------------ surrogate (linear-basis) form
// z_b = sum_lm c_lm,b(lambda) -2Y_lm(iota, phi) per joint sample (rows 0..6
// extrinsic, row 7 lambda of smp [8][N]); gp holds the physical modes' Y
// tables; A [n_lm][n_b][n_pow] complex; err bit 0 for lambda outside [-1, 1]
// (z = NaN).
hipError_t ile_launch_rom_z(const ile_geom &gp, const double *smp, int64_t N, const double *A,
                            int n_b, int n_pow, double *Z, int32_t *err, hipStream_t st);

// ------------------------------------ Q, U, V from the frequency domain
// prod: X [n_det][n_lm][n] complex; err bit 0 for a non-finite input or a
// non-positive spectrum in the band.  ifft_rows: inverse FFT of `rows`
// complex rows of n (power of two) ping-ponging between a (input) and b;
// *result is the buffer holding the output.
hipError_t ile_launch_fd_prod(const double *h, const double *d, const double *psd, int64_t n,
                              int n_det, int n_lm, double df, double f_min, double f_max,
                              double t0, double *X, int32_t *err, hipStream_t st);
int ile_fft_passes(int64_t n);
hipError_t ile_launch_ifft_rows(double *a, double *b, int64_t n, int rows, double **result,
                                hipStream_t st);
hipError_t ile_launch_uv_fd(const double *h, const double *psd, int64_t n, int n_det, int n_lm,
                            double df, double f_min, double f_max, double *U, double *V,
                            hipStream_t st);

// ------------------------------------------------ extrinsic harvest
// weights: w = exp(ln w - max ln w), ln w = lnL + ln p - ln q (NULL: 0),
// part: ile_hv_parts() + 1 doubles; err bit 0: an invalid ln p / ln q, bit 1:
// no finite positive weight.  pick (u is [2][n_out]): err bit 2 for a uniform
// outside [0, 1) in either row.
int ile_hv_parts();
hipError_t ile_launch_hv_weights(const double *lnL, const double *ln_p, const double *ln_q,
                                 int64_t n, double *w, double *part, int32_t *err,
                                 hipStream_t st);
hipError_t ile_launch_hv_pick(const double *cdf, int64_t n, const double *u, int64_t n_out,
                              int64_t *idx, int32_t *err, hipStream_t st);
hipError_t ile_launch_hv_gather(const double *smp, int64_t ld, const int64_t *idx, int64_t m,
                                double *sel, hipStream_t st);
// one wave per row of series[m][n_t]; theta [7][ld_out] may be NULL
hipError_t ile_launch_hv_bin(const double *series, int64_t m, int n_t, const double *v,
                             const double *sel, double srate, int32_t *bins, double *theta,
                             int64_t ld_out, hipStream_t st);

// ------------------------------------------------ learned proposal (MDN)
// Network sizes and the flat parameter layout (W1 | b1 | W2 | b2 | W3 | b3,
// row-major, masked entries held at zero) documented in ile.h.
#define ILE_MDN_D 7
#define ILE_MDN_H 128
#define ILE_MDN_C 16
#define ILE_MDN_O 336
#define ILE_MDN_OFF_W1 0
#define ILE_MDN_OFF_B1 896
#define ILE_MDN_OFF_W2 1024
#define ILE_MDN_OFF_B2 17408
#define ILE_MDN_OFF_W3 17536
#define ILE_MDN_OFF_B3 60544
#define ILE_MDN_NPARAM 60880
#define ILE_MDN_W3T_LD 384    // rows of the transposed W3 copy, zero past 336
#define ILE_MDN_NPART 60928   // per-workgroup partial: grads, loss sum, weight sum
#define ILE_MDN_TILE 64       // samples per workgroup pass

// MADE masks: hidden unit k has degree k mod 6; unit k sees inputs
// i <= deg(k); layer-2 unit k2 sees k1 with deg(k1) <= deg(k2); output o
// (dimension o / 48) sees units with deg(k) < o / 48.  Biases are free.
__host__ __device__ inline bool ile_mdn_trainable(int j)
{
    if (j < 0 || j >= ILE_MDN_NPARAM) return false;
    if (j < ILE_MDN_OFF_B1) return (j % ILE_MDN_D) <= (j / ILE_MDN_D) % 6;
    if (j < ILE_MDN_OFF_W2) return true;
    if (j < ILE_MDN_OFF_B2) {
        const int q = j - ILE_MDN_OFF_W2;
        return (q % ILE_MDN_H) % 6 <= (q / ILE_MDN_H) % 6;
    }
    if (j < ILE_MDN_OFF_W3) return true;
    if (j < ILE_MDN_OFF_B3) {
        const int q = j - ILE_MDN_OFF_W3;
        return (q % ILE_MDN_H) % 6 < (q / ILE_MDN_H) / (3 * ILE_MDN_C);
    }
    return true;
}

// Transform between the sample vector and the network's inputs.
struct ile_mdn_tr {
    double origin[3];   // ra, psi, phi origins
    double mean[7], scale[7];
    double d_min, d_max, t_ref_max, sigma_floor;
    double sigma_scale;   // kappa of draws and densities (training: 1)
};

// Device state of one proposal.
struct ile_mdn_dev {
    float *theta, *m, *v;               // [NPARAM] master weights and Adam moments
    __bf16 *W2b, *W3b;                  // [o][k] copies (forward operands)
    __bf16 *W2t, *W3t;                  // [k][o] copies (backward operands)
    ile_mdn_tr *tr;                     // transform
};

// Defensive mixture with the histogram proposal (nb = 0 or eps = 0: none).
struct ile_mdn_mix {
    int nb;
    const double *P, *C;   // histogram state [2][nb], [2][nb+1]
    double eps;
};

hipError_t ile_launch_mdn_cast(const ile_mdn_dev &M, hipStream_t st);
// ln q of n samples x[7][ld] (optionally mixed), or draws of n samples
// (counters first..first+n-1 of key seed) with their ln p and ln q.
hipError_t ile_launch_mdn_logpdf(const ile_mdn_dev &M, const ile_mdn_mix &mix,
                                 const double *x, int64_t ld, int64_t n, double *ln_q,
                                 int grid, hipStream_t st);
hipError_t ile_launch_mdn_sample(const ile_mdn_dev &M, const ile_mdn_mix &mix,
                                 uint64_t seed, int64_t first, int64_t n, double *x,
                                 int64_t ld, double *ln_p, double *ln_q, int grid,
                                 hipStream_t st);
// Training pieces.  prepare: z~ and tempered weights; cdf: inclusive
// prefix sums of the weights.
// fit: tempering (ESS target ess_frac of the finite samples) into stats =
// {max ln w, beta}, and (if fit_transform) the transform into tr; ws is a
// workspace of ile_mdn_fit_ws_doubles() doubles.
hipError_t ile_launch_mdn_fit(const double *x, int64_t ld, const double *lnw, int64_t n,
                              double ess_frac, ile_mdn_tr *tr, double *stats, double *ws,
                              bool fit_transform, hipStream_t st);
size_t ile_mdn_fit_ws_doubles();
hipError_t ile_launch_mdn_prepare(const ile_mdn_tr *tr, const double *x, int64_t ld,
                                  const double *lnw, int64_t n, const double *stats,
                                  float *z, double *w, hipStream_t st);
// the same with given weights w_in (NULL: 1) instead of tempered ones
hipError_t ile_launch_mdn_prepare_w(const ile_mdn_tr *tr, const double *x, int64_t ld,
                                    const double *w_in, int64_t n, float *z, double *w,
                                    hipStream_t st);
hipError_t ile_launch_mdn_cdf(const double *w, int64_t n, double *cdf, double *ws,
                              hipStream_t st);   // ws: ile_mdn_fit_ws_doubles() doubles
// count minibatch draws (index i with probability w_i / sum w), Philox
// counters (draw, 0, 0x4D444E54) of key seed
hipError_t ile_launch_mdn_draw_idx(uint64_t seed, int64_t count, const double *cdf, int64_t n,
                                   int32_t *idx, hipStream_t st);
// Forward + backward of a batch: per-workgroup partials [grid][NPART].
hipError_t ile_launch_mdn_grad(const ile_mdn_dev &M, const float *z, int64_t ldz,
                               const int32_t *idx, const double *w, int batch, float *part,
                               hipStream_t st);
// Reduce the partials in fixed order; mask; write the gradient (grad may be
// NULL) and the loss; if adam, take one Adam step number `step` (1-based).
hipError_t ile_launch_mdn_update(const ile_mdn_dev &M, const float *part, int n_part,
                                 float *grad, double *loss, bool adam, int64_t step, double lr,
                                 hipStream_t st);
hipError_t ile_launch_lnw(const double *lnL, const double *ln_p, const double *ln_q, int64_t n,
                          double *lnw, hipStream_t st);

// cross-object accessors (defined in ile_api.cpp / ile_prop_api.cpp)
hipStream_t ile_ctx_stream(const ile_ctx *c);
int ile_ctx_hist(const ile_ctx *c, const double **P, const double **C);   // nb, or 0
const ile_mdn_dev &ile_prop_dev(const ile_prop *p);
hipStream_t ile_prop_stream(const ile_prop *p);
int ile_prop_grid(const ile_prop *p);

// Zero-noise injection (ile_kernels.hip): detector responses d[n_det][n] of
// theta (device, 7 doubles), then Q [n_det][n_lm][n] (scaled), U and V
// [n_lm][n_lm] (complex interleaved).
hipError_t ile_launch_inject(const ile_geom &g, const double *h, int n, const double *theta,
                             double *d, hipStream_t st);
hipError_t ile_launch_inject_qv(int n_det, int n_lm, int n, const double *h, const double *d,
                                double scale, double *Q, double *U, double *V, hipStream_t st);
