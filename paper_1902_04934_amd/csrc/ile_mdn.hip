// ile_mdn.hip -- the learned proposal: a masked autoregressive mixture
// density network over the 7 extrinsic parameters, on the matrix cores.
//
// The paper draws its Monte Carlo samples from an adaptive proposal built
// from one-dimensional histograms (Sec. II.A, Sec. III.C); this network is a
// richer proposal trained on the weighted samples of the first adaptive
// rounds, used in a defensive mixture with the histogram proposal.
//
// Model (parameter layout in ile.h): inputs z~[7] (the transformed sample),
// h1 = tanh(W1 z~ + b1), h2 = tanh(W2 h1 + b2), o = W3 h2 + b3, with MADE
// masks (hidden degree k mod 6) so that dimension d's 16-component Gaussian
// mixture, o[48d .. 48d+47] = (logits, means, scale pre-activations),
// depends on z~_0..z~_{d-1} only.
//
// Arithmetic: layer 1 (7 inputs) in FP32 on the vector ALUs; layers 2 and 3
// on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation); mixture
// densities in FP32; the transform, its Jacobian, ln p and the mixture with
// the histogram proposal in FP64.  One wave evaluates 16 samples: lane
// l = 16 g + r holds sample r's inputs (A layout: row r, k = 8 g .. 8 g + 7
// of each 32-wide K step) and receives outputs for samples 4 g + v, v < 4,
// at column r (D layout); a sample's 16 mixture components therefore sit
// in one 16-lane group and its log-sum-exps are 16-lane butterflies.
//
// Training: each workgroup runs forward and backward for 64 samples and
// writes its gradient as one partial row; a second kernel sums the rows in
// a fixed order and takes the Adam step, so training is bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ile_internal.h"
#include "ile_rng.h"

namespace {

constexpr int D = ILE_MDN_D, H = ILE_MDN_H, O = ILE_MDN_O;
constexpr int OFF_W1 = ILE_MDN_OFF_W1, OFF_B1 = ILE_MDN_OFF_B1, OFF_W2 = ILE_MDN_OFF_W2,
              OFF_B2 = ILE_MDN_OFF_B2, OFF_W3 = ILE_MDN_OFF_W3, OFF_B3 = ILE_MDN_OFF_B3,
              NPARAM = ILE_MDN_NPARAM, NPART = ILE_MDN_NPART, W3T_LD = ILE_MDN_W3T_LD;
constexpr int WLD = 136;   // LDS row of a [row][128] bf16 array (+16 bytes: no bank conflicts)
constexpr int SLD = 72;    // LDS row of a [unit][64 samples] bf16 array
constexpr int CLD = 104;   // LDS row of a 96-output chunk of dL/do
constexpr int MAXB = 64;   // histogram bins held in LDS
constexpr double kPi = 3.141592653589793238463;
constexpr double kTwoPi = 6.283185307179586476925;
constexpr float kHalfLn2Pi = 0.91893853320467274178f;

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4f mfma(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline float softplusf(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }

// Branch-free functions at the hardware's transcendental rate for the
// training gradient (a few ulp; the BF16 operands of the products dominate
// its error).  exp and log through the base-2 instructions.
__device__ inline float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ inline float flog(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// tanh: odd Taylor series through x^9 for |x| < 0.2 (truncation < 1e-9
// relative), else (1 - e) / (1 + e) with e = exp(-2|x|)
__device__ inline float ftanh(float x)
{
    const float ax = fabsf(x), x2 = x * x;
    const float poly = ax + ax * x2 * (-1.f / 3.f + x2 * (2.f / 15.f + x2 * (-17.f / 315.f +
                                                                        x2 * (62.f / 2835.f))));
    const float e = fexp(-2.f * ax);
    const float big = (1.f - e) * frcp(1.f + e);
    return copysignf(ax < 0.2f ? poly : big, x);
}
__device__ inline float fsoftplus(float x) { return fmaxf(x, 0.f) + flog(1.f + fexp(-fabsf(x))); }
__device__ inline float fsigmoid(float x) { return frcp(1.f + fexp(-x)); }

// 16-lane reductions by DPP rotations within a row (8, 4, 2, 1 lanes):
// after the rotation by n the partial values repeat with period n, so
// lane i meets the same partner value as in an xor butterfly, and every
// lane of the group ends with the same bits (each step combines the same
// two operands in either order).  DPP moves data between lanes in the
// VALU, without the LDS round trip of a permute.
template <int N>
__device__ inline float row_ror(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        0, __builtin_bit_cast(int, x), 0x120 + N, 0xF, 0xF, false));
}
__device__ inline float gmax(float x)
{
    x = fmaxf(x, row_ror<8>(x));
    x = fmaxf(x, row_ror<4>(x));
    x = fmaxf(x, row_ror<2>(x));
    return fmaxf(x, row_ror<1>(x));
}
__device__ inline float gsum(float x)
{
    x += row_ror<8>(x);
    x += row_ror<4>(x);
    x += row_ror<2>(x);
    return x + row_ror<1>(x);
}

// Ordering point for LDS data handed between lanes of one wave: a wave's
// LDS accesses are performed in issue order, so it is enough that the
// compiler moves no access across this point (no workgroup barrier).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ transform
// u in (0,1) of dimension d and ln |du/dx|
__device__ inline double to_unit(const ile_mdn_tr &T, int d, double x, double &ldu)
{
    double y;
    switch (d) {
    case 0:
        y = (x - T.origin[0]) / kTwoPi + 0.5;
        ldu = -log(kTwoPi);
        return y - floor(y);
    case 1:
        ldu = log(cos(x) / 2.0);
        return (sin(x) + 1.0) / 2.0;
    case 2:
        y = (x - T.origin[1]) / kPi + 0.5;
        ldu = -log(kPi);
        return y - floor(y);
    case 3:
        y = (x - T.origin[2]) / kTwoPi + 0.5;
        ldu = -log(kTwoPi);
        return y - floor(y);
    case 4:
        ldu = -log(2.0);
        return (x + 1.0) / 2.0;
    case 5:
        ldu = -log(T.d_max - T.d_min);
        return (x - T.d_min) / (T.d_max - T.d_min);
    default:
        ldu = -log(2.0 * T.t_ref_max);
        return (x + T.t_ref_max) / (2.0 * T.t_ref_max);
    }
}

// inverse of to_unit; periodic parameters wrapped into their prior range
__device__ inline double from_unit(const ile_mdn_tr &T, int d, double u)
{
    double x;
    switch (d) {
    case 0:
        x = T.origin[0] + (u - 0.5) * kTwoPi;
        return x - kTwoPi * floor(x / kTwoPi);
    case 1: return asin(2.0 * u - 1.0);
    case 2:
        x = T.origin[1] + (u - 0.5) * kPi;
        return x - kPi * floor(x / kPi);
    case 3:
        x = T.origin[2] + (u - 0.5) * kTwoPi;
        return x - kTwoPi * floor(x / kTwoPi);
    case 4: return 2.0 * u - 1.0;
    case 5: return T.d_min + u * (T.d_max - T.d_min);
    default: return (2.0 * u - 1.0) * T.t_ref_max;
    }
}

// x -> z~ (FP32 network inputs); returns sum_d ln |dz~_d/dx_d|, or -inf when
// a u is 0 or 1 (z~ is then 0 in that dimension)
__device__ inline double to_z(const ile_mdn_tr &T, const double x[7], float z[7])
{
    double lj = 0.0;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; d++) {
        double ldu;
        const double u = to_unit(T, d, x[d], ldu);
        if (!(u > 0.0 && u < 1.0)) {
            ok = false;
            z[d] = 0.f;
            continue;
        }
        const double lu = log(u), l1u = log1p(-u);
        z[d] = (float)((lu - l1u - T.mean[d]) / T.scale[d]);
        lj += -log(T.scale[d]) - lu - l1u + ldu;
    }
    return ok ? lj : -INFINITY;
}

__device__ inline double logaddexp(double a, double b)
{
    const double m = fmax(a, b);
    if (m == -INFINITY) return -INFINITY;
    return m + log(exp(a - m) + exp(b - m));
}

// ln (q_hist / p) of the histogram proposal at (ra, dec)
__device__ inline double ln_hist_ratio(const double *P, int nb, double ra, double dec)
{
    int br = (int)floor(ra * (nb / kTwoPi));
    int bs = (int)floor((sin(dec) + 1.0) * (0.5 * nb));
    br = min(max(br, 0), nb - 1);
    bs = min(max(bs, 0), nb - 1);
    return log(nb * P[br]) + log(nb * P[nb + bs]);
}

// ---------------------------------------------------------- the layers
// Layer 1 for sample r: units k = 32 ks + 8 g + i as BF16 A fragments.
template <bool FAST = false>
__device__ inline void layer1(const float *W1, int w1ld, const float *b1, const float z[7],
                              int g, v8bf A[4])
{
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int k = 32 * ks + 8 * g + i;
            float a = b1[k];
#pragma unroll
            for (int d = 0; d < D; d++) a = fmaf(W1[k * w1ld + d], z[d], a);
            A[ks][i] = (__bf16)(FAST ? ftanh(a) : tanhf(a));
        }
    }
}

// Pre-activations of layer 2: acc[t][v] = a2[sample 4g+v][unit 16t+r].
// W2 is [o][k] with row stride ld (LDS or global).
__device__ inline void layer2(const v8bf A[4], const __bf16 *W2, int ld, int r, int g,
                              v4f acc[8])
{
#pragma unroll
    for (int t = 0; t < 8; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const v8bf b = *(const v8bf *)(W2 + (16 * t + r) * ld + 32 * ks + 8 * g);
            acc[t] = mfma(A[ks], b, acc[t]);
        }
    }
}

// B fragments of the three layer-3 output tiles of dimension d, [4 ks][3 j].
__device__ inline void load_w3_dim(const __bf16 *W3, int ld, int d, int r, int g, v8bf B[12])
{
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            B[3 * ks + j] = *(const v8bf *)(W3 + (48 * d + 16 * j + r) * ld + 32 * ks + 8 * g);
}

// Three output tiles 3d, 3d+1, 3d+2 (dimension d) of layer 3.
__device__ inline void layer3_dim(const v8bf A2[4], const __bf16 *W3, int ld, int d, int r,
                                  int g, v4f t3[3])
{
#pragma unroll
    for (int j = 0; j < 3; j++) t3[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const v8bf b = *(const v8bf *)(W3 + (48 * d + 16 * j + r) * ld + 32 * ks + 8 * g);
            t3[j] = mfma(A2[ks], b, t3[j]);
        }
    }
}

// ln q_d of one sample from its component (lane r of the group): returns
// the log density; sig, rr = (z - mu)/sig, ell = log weight + log normal
// of this component, la = log-sum-exp of the logits.
__device__ inline float mix_lnq(float a, float mu, float rho, float z, float sfloor, float kappa,
                                float &sig, float &rr, float &ell, float &la)
{
    const float ma = gmax(a);
    la = ma + logf(gsum(expf(a - ma)));
    sig = kappa * (sfloor + softplusf(rho));
    rr = (z - mu) / sig;
    ell = a - la - 0.5f * rr * rr - logf(sig) - kHalfLn2Pi;
    const float ml = gmax(ell);
    return ml + logf(gsum(expf(ell - ml)));
}

// mix_lnq with the branch-free functions (training gradient); rs = 1/sig
__device__ inline float mix_lnq_fast(float a, float mu, float rho, float z, float sfloor,
                                     float &rs, float &rr, float &ell, float &la)
{
    const float ma = gmax(a);
    la = ma + flog(gsum(fexp(a - ma)));
    const float sig = sfloor + fsoftplus(rho);
    rs = frcp(sig);
    rr = (z - mu) * rs;
    ell = a - la - 0.5f * rr * rr - flog(sig) - kHalfLn2Pi;
    const float ml = gmax(ell);
    return ml + flog(gsum(fexp(ell - ml)));
}

// ----------------------------------------------------------- inference
// Persistent: each workgroup stages the BF16 weights in LDS once and loops
// over tiles of 64 samples (4 waves x 16).  SAMPLE: ancestral draw of z~,
// one dimension per pass, then the density of the drawn x by the same code
// as LOGPDF, so the returned ln q is exactly what logpdf gives for it.
template <bool SAMPLE>
__global__ __launch_bounds__(256) void k_mdn_infer(
    const float *__restrict__ theta, const __bf16 *__restrict__ W2b,
    const __bf16 *__restrict__ W3b, const ile_mdn_tr *__restrict__ trp, ile_mdn_mix mix,
    uint64_t seed, int64_t first, int64_t n, double *x_io, int64_t ld, double *ln_p,
    double *ln_q)
{
    __shared__ __attribute__((aligned(16))) __bf16 sW2[H * WLD];
    __shared__ __attribute__((aligned(16))) __bf16 sW3[O * WLD];
    __shared__ float sW1[H * 8];
    __shared__ float sb1[H], sb2[H], sb3[O];
    __shared__ __attribute__((aligned(16))) __bf16 sH[4][16 * WLD];
    __shared__ float sZ[4][16 * 8];
    __shared__ float sR[4][16 * 16];
    __shared__ float sLq[4][16];
    __shared__ double sP[2 * MAXB], sC[2 * (MAXB + 1)];
    __shared__ ile_mdn_tr sT;

    const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int c = tid; c < H * 16; c += 256) {
        const int row = c >> 4, col = c & 15;
        *(v8bf *)(sW2 + row * WLD + 8 * col) = *(const v8bf *)(W2b + row * H + 8 * col);
    }
    for (int c = tid; c < O * 16; c += 256) {
        const int row = c >> 4, col = c & 15;
        *(v8bf *)(sW3 + row * WLD + 8 * col) = *(const v8bf *)(W3b + row * H + 8 * col);
    }
    for (int j = tid; j < H * 8; j += 256) {
        const int k = j >> 3, d = j & 7;
        sW1[j] = d < D ? theta[OFF_W1 + k * D + d] : 0.f;
    }
    for (int j = tid; j < H; j += 256) {
        sb1[j] = theta[OFF_B1 + j];
        sb2[j] = theta[OFF_B2 + j];
    }
    for (int j = tid; j < O; j += 256) sb3[j] = theta[OFF_B3 + j];
    const bool mixed = mix.nb > 0 && mix.eps > 0.0;
    if (mixed) {
        for (int j = tid; j < 2 * mix.nb; j += 256) sP[j] = mix.P[j];
        for (int j = tid; j < 2 * (mix.nb + 1); j += 256) sC[j] = mix.C[j];
    }
    if (tid == 0) sT = *trp;
    __syncthreads();
    const float sfloor = (float)sT.sigma_floor, kappa = (float)sT.sigma_scale;
    __bf16 *Hs = sH[w];
    float *Zs = sZ[w], *Rs = sR[w];

    for (int64_t tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
        const int64_t i = tile * 64 + 16 * w + r;   // sample of lane r (group 0 owns it)
        const bool valid = i < n;
        double x[7] = {1.0, 0.1, 1.0, 1.0, 0.1, 0.5 * (sT.d_min + sT.d_max), 0.0};
        if (SAMPLE) {
            // 16 uniforms per sample: group g computes Philox blocks 2g, 2g+1
#pragma unroll
            for (int bb = 0; bb < 2; bb++) {
                uint32_t q[4];
                ile_rng::block(seed, (uint64_t)(first + i), 2 * g + bb, ile_rng::kTagMdn, q);
                Rs[r * 16 + 4 * g + 2 * bb] = (float)ile_rng::u53(q[0], q[1]);
                Rs[r * 16 + 4 * g + 2 * bb + 1] = (float)ile_rng::u53(q[2], q[3]);
            }
            if (g == 0)
                for (int d = 0; d < 8; d++) Zs[r * 8 + d] = 0.f;
            __syncthreads();
            // uniforms 0..6: component choices; 7..14 -> 8 normals (Box-Muller);
            // 15: which member of the defensive mixture draws the sample
            if (g == 0) {
                for (int j = 0; j < 4; j++) {
                    const float a = Rs[r * 16 + 7 + 2 * j], b = Rs[r * 16 + 8 + 2 * j];
                    const float rad = sqrtf(-2.f * logf(a));
                    float sn, cs;
                    sincosf(6.28318530717958648f * b, &sn, &cs);
                    Rs[r * 16 + 7 + 2 * j] = rad * cs;
                    Rs[r * 16 + 8 + 2 * j] = rad * sn;
                }
            }
            __syncthreads();
            for (int d = 0; d < D; d++) {
                v4f t3[3];
                if (d > 0) {
                    float z[7];
#pragma unroll
                    for (int e = 0; e < D; e++) z[e] = Zs[r * 8 + e];
                    v8bf A1[4];
                    layer1(sW1, 8, sb1, z, g, A1);
                    v4f acc[8];
                    layer2(A1, sW2, WLD, r, g, acc);
#pragma unroll
                    for (int t = 0; t < 8; t++) {
                        const float bb = sb2[16 * t + r];
#pragma unroll
                        for (int v = 0; v < 4; v++)
                            Hs[(4 * g + v) * WLD + 16 * t + r] = (__bf16)tanhf(acc[t][v] + bb);
                    }
                    __syncthreads();
                    v8bf A2[4];
#pragma unroll
                    for (int ks = 0; ks < 4; ks++)
                        A2[ks] = *(const v8bf *)(Hs + r * WLD + 32 * ks + 8 * g);
                    layer3_dim(A2, sW3, WLD, d, r, g, t3);
                } else {
                    // dimension 0 sees no hidden unit: its outputs are the biases
#pragma unroll
                    for (int j = 0; j < 3; j++) t3[j] = v4f{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int s = 4 * g + v;
                    const float al = t3[0][v] + sb3[48 * d + r];
                    const float mu = t3[1][v] + sb3[48 * d + 16 + r];
                    const float rho = t3[2][v] + sb3[48 * d + 32 + r];
                    // categorical draw: first component whose cumulative weight
                    // exceeds u times the total
                    const float ma = gmax(al);
                    float cum = expf(al - ma);
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) {
                        const float tt = __shfl_up(cum, off, 16);
                        if (r >= off) cum += tt;
                    }
                    const float tot = __shfl(cum, 15, 16);
                    const unsigned long long bal = __ballot(cum > Rs[s * 16 + d] * tot);
                    const unsigned bits = (unsigned)(bal >> (16 * g)) & 0xffffu;
                    const int cs = bits ? __ffs(bits) - 1 : 15;
                    const float sig = kappa * (sfloor + softplusf(rho));
                    const float mus = __shfl(mu, cs, 16), sgs = __shfl(sig, cs, 16);
                    if (r == 0) Zs[s * 8 + d] = mus + sgs * Rs[s * 16 + 7 + d];
                }
                __syncthreads();
            }
            if (g == 0) {
                if (mixed && Rs[r * 16 + 15] < (float)mix.eps) {
                    uint32_t wd[16];
                    ile_rng::prior_words(seed, (uint64_t)(first + i), wd);
                    int br, bs;
                    (void)ile_rng::hist_sample(sP, sC, mix.nb, wd, sT.d_min, sT.d_max,
                                               sT.t_ref_max, x, br, bs);
                } else {
                    for (int d = 0; d < D; d++) {
                        const double zz = sT.mean[d] + sT.scale[d] * (double)Zs[r * 8 + d];
                        x[d] = from_unit(sT, d, 1.0 / (1.0 + exp(-zz)));
                    }
                }
            }
        } else if (g == 0 && valid) {
            for (int d = 0; d < D; d++) x[d] = x_io[d * ld + i];
        }
        // ---- density of x: the same code in both modes
        double jac = 0.0, lp = 0.0, lqa = 0.0;
        if (g == 0) {
            float z[7];
            jac = to_z(sT, x, z);
            for (int d = 0; d < D; d++) Zs[r * 8 + d] = z[d];
            lp = ile_rng::ln_prior(x[1], x[5], sT.d_min, sT.d_max, sT.t_ref_max);
            if (mixed) lqa = lp + ln_hist_ratio(sP, mix.nb, x[0], x[1]);
        }
        __syncthreads();
        {
            float z[7];
#pragma unroll
            for (int e = 0; e < D; e++) z[e] = Zs[r * 8 + e];
            v8bf A1[4];
            layer1(sW1, 8, sb1, z, g, A1);
            v4f acc[8];
            layer2(A1, sW2, WLD, r, g, acc);
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const float bb = sb2[16 * t + r];
#pragma unroll
                for (int v = 0; v < 4; v++)
                    Hs[(4 * g + v) * WLD + 16 * t + r] = (__bf16)tanhf(acc[t][v] + bb);
            }
            __syncthreads();
            v8bf A2[4];
#pragma unroll
            for (int ks = 0; ks < 4; ks++) A2[ks] = *(const v8bf *)(Hs + r * WLD + 32 * ks + 8 * g);
            float lqz[4] = {0.f, 0.f, 0.f, 0.f};
            for (int d = 0; d < D; d++) {
                v4f t3[3];
                layer3_dim(A2, sW3, WLD, d, r, g, t3);
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    float sig, rr, ell, la;
                    lqz[v] += mix_lnq(t3[0][v] + sb3[48 * d + r], t3[1][v] + sb3[48 * d + 16 + r],
                                      t3[2][v] + sb3[48 * d + 32 + r], Zs[(4 * g + v) * 8 + d],
                                      sfloor, kappa, sig, rr, ell, la);
                }
            }
            if (r == 0)
                for (int v = 0; v < 4; v++) sLq[w][4 * g + v] = lqz[v];
        }
        __syncthreads();
        if (g == 0 && valid) {
            const double lnn = jac == -INFINITY ? -INFINITY : (double)sLq[w][r] + jac;
            double lq = mixed ? logaddexp(log1p(-mix.eps) + lnn, log(mix.eps) + lqa) : lnn;
            if (SAMPLE) {
                // a draw on the boundary of the support (probability 0) has
                // p = 0: a finite ln q makes its weight exactly 0
                if (!(lp > -INFINITY) || !(lq > -INFINITY)) lq = 0.0;
                for (int d = 0; d < D; d++) x_io[d * ld + i] = x[d];
                if (ln_p) ln_p[i] = lp;
            }
            ln_q[i] = lq;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ training
// Forward and backward of 64 samples (batch slots blockIdx.x*64 ..): the
// workgroup's gradient of  L = -sum_s w_s ln q(z~_s)  (not yet divided by
// sum w), its loss sum and weight sum go to part[blockIdx.x][.].
__global__ __launch_bounds__(256) void k_mdn_grad(
    const float *__restrict__ theta, const __bf16 *__restrict__ W2b,
    const __bf16 *__restrict__ W3b, const __bf16 *__restrict__ W2t,
    const __bf16 *__restrict__ W3t, const ile_mdn_tr *__restrict__ trp,
    const float *__restrict__ zt, int64_t ldz, const int32_t *__restrict__ idx,
    const double *__restrict__ wts, int batch, float *__restrict__ part)
{
    __shared__ float sZ[64 * 8];
    __shared__ float sWt[64];
    __shared__ __attribute__((aligned(16))) __bf16 sH1T[H * SLD];    // h1 [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sH2T[H * SLD];    // h2 [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sDOT[O * SLD];    // dL/do [output][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sDA2T[H * SLD];   // dL/da2 [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sDA1T[H * SLD];   // dL/da1 [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sHs[4][16 * WLD]; // per wave: h2, then dL/da2 [s][unit]
    __shared__ __attribute__((aligned(16))) __bf16 sDOc[4][16 * CLD];// per wave: 96 outputs of dL/do [s][o]
    __shared__ float sLoss[4];
    __shared__ float sPar[OFF_W2 + H + O];   // FP32 W1, b1, b2, b3

    const float *W1 = sPar, *b1 = sPar + OFF_B1, *b2 = sPar + OFF_W2,
                *b3 = sPar + OFF_W2 + H;
    const float sfloor = (float)trp->sigma_floor;
    const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s0 = 16 * w;
    __bf16 *Hs = sHs[w], *DOc = sDOc[w];

    // layer-2 fragments first: their loads overlap the staging below
    v8bf B2f[32];
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int t = 0; t < 8; t++)
            B2f[8 * ks + t] = *(const v8bf *)(W2b + (16 * t + r) * H + 32 * ks + 8 * g);
    if (g == 0) {
        const int64_t b = (int64_t)blockIdx.x * 64 + s0 + r;
        const bool valid = b < batch;
        const int64_t row = valid ? (idx ? (int64_t)idx[b] : b) : 0;
        for (int d = 0; d < 8; d++) sZ[(s0 + r) * 8 + d] = (valid && d < D) ? zt[d * ldz + row] : 0.f;
        sWt[s0 + r] = valid ? (wts ? (float)wts[row] : 1.f) : 0.f;
    }
    for (int e = tid; e < OFF_W2 + H + O; e += 256)
        sPar[e] = e < OFF_W2 ? theta[OFF_W1 + e]
                : e < OFF_W2 + H ? theta[OFF_B2 + e - OFF_W2] : theta[OFF_B3 + e - OFF_W2 - H];
    __syncthreads();

    // ---- forward
    v8bf A1[4];
    {
        float z[7];
#pragma unroll
        for (int d = 0; d < D; d++) z[d] = sZ[(s0 + r) * 8 + d];
        layer1<true>(W1, D, b1, z, g, A1);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int i = 0; i < 8; i++) sH1T[(32 * ks + 8 * g + i) * SLD + s0 + r] = A1[ks][i];
    float h2v[8][4];
    {
        v4f acc[8];
#pragma unroll
        for (int t = 0; t < 8; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
#pragma unroll
            for (int t = 0; t < 8; t++) acc[t] = mfma(A1[ks], B2f[8 * ks + t], acc[t]);
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const float bb = b2[16 * t + r];
            v4bf pk;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const float h = ftanh(acc[t][v] + bb);
                h2v[t][v] = h;
                pk[v] = (__bf16)h;
                Hs[(4 * g + v) * WLD + 16 * t + r] = pk[v];
            }
            *(v4bf *)(sH2T + (16 * t + r) * SLD + s0 + 4 * g) = pk;
        }
    }
    wave_lds_sync();   // Hs is the wave's own; sH2T is read after later barriers
    v8bf A2[4];
#pragma unroll
    for (int ks = 0; ks < 4; ks++) A2[ks] = *(const v8bf *)(Hs + r * WLD + 32 * ks + 8 * g);

    // ---- layer 3, mixture gradients and dL/dh2, two dimensions at a time.
    // The W3 fragments of the next dimension and the W3^T fragments of the
    // current pair are loaded ahead of the arithmetic that needs them.
    v4f dh2[8];
#pragma unroll
    for (int t = 0; t < 8; t++) dh2[t] = v4f{0.f, 0.f, 0.f, 0.f};
    float lacc = 0.f;
    v8bf Bn[12];
    load_w3_dim(W3b, H, 0, r, g, Bn);
#pragma unroll 1
    for (int p = 0; p < 4; p++) {
        v8bf Bt[24];
#pragma unroll
        for (int ks = 0; ks < 3; ks++)
#pragma unroll
            for (int t = 0; t < 8; t++)
                Bt[8 * ks + t] = *(const v8bf *)(W3t + (16 * t + r) * W3T_LD + 96 * p + 32 * ks + 8 * g);
#pragma unroll
        for (int dd = 0; dd < 2; dd++) {
            const int d = 2 * p + dd;
            if (d < D) {
                v8bf Bc[12];
#pragma unroll
                for (int j = 0; j < 12; j++) Bc[j] = Bn[j];
                if (d + 1 < D) load_w3_dim(W3b, H, d + 1, r, g, Bn);
                v4f t3[3];
#pragma unroll
                for (int j = 0; j < 3; j++) t3[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ks++)
#pragma unroll
                    for (int j = 0; j < 3; j++) t3[j] = mfma(A2[ks], Bc[3 * ks + j], t3[j]);
                v4bf ga, gm, gr;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int s = 4 * g + v;
                    const float al = t3[0][v] + b3[48 * d + r];
                    const float mu = t3[1][v] + b3[48 * d + 16 + r];
                    const float rho = t3[2][v] + b3[48 * d + 32 + r];
                    const float ws = sWt[s0 + s];
                    float rs, rr, ell, la;
                    const float lq = mix_lnq_fast(al, mu, rho, sZ[(s0 + s) * 8 + d], sfloor, rs, rr, ell, la);
                    const float gam = fexp(ell - lq), pi = fexp(al - la);
                    if (r == 0) lacc -= ws * lq;
                    ga[v] = (__bf16)(-ws * (gam - pi));
                    gm[v] = (__bf16)(-ws * gam * rr * rs);
                    gr[v] = (__bf16)(-ws * gam * (rr * rr - 1.f) * rs * fsigmoid(rho));
                    DOc[s * CLD + 48 * dd + r] = ga[v];
                    DOc[s * CLD + 48 * dd + 16 + r] = gm[v];
                    DOc[s * CLD + 48 * dd + 32 + r] = gr[v];
                }
                *(v4bf *)(sDOT + (48 * d + r) * SLD + s0 + 4 * g) = ga;
                *(v4bf *)(sDOT + (48 * d + 16 + r) * SLD + s0 + 4 * g) = gm;
                *(v4bf *)(sDOT + (48 * d + 32 + r) * SLD + s0 + 4 * g) = gr;
            } else {
#pragma unroll
                for (int v = 0; v < 4; v++)
#pragma unroll
                    for (int j = 0; j < 3; j++) DOc[(4 * g + v) * CLD + 48 * dd + 16 * j + r] = (__bf16)0.f;
            }
        }
        wave_lds_sync();   // DOc is the wave's own
#pragma unroll
        for (int ks = 0; ks < 3; ks++) {
            const v8bf a = *(const v8bf *)(DOc + r * CLD + 32 * ks + 8 * g);
#pragma unroll
            for (int t = 0; t < 8; t++) dh2[t] = mfma(a, Bt[8 * ks + t], dh2[t]);
        }
        wave_lds_sync();
    }

    // ---- dL/da2 = dL/dh2 (1 - h2^2)
    v8bf B2[32];
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int t = 0; t < 8; t++)
            B2[8 * ks + t] = *(const v8bf *)(W2t + (16 * t + r) * H + 32 * ks + 8 * g);
#pragma unroll
    for (int t = 0; t < 8; t++) {
        v4bf pk;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            pk[v] = (__bf16)(dh2[t][v] * (1.f - h2v[t][v] * h2v[t][v]));
            Hs[(4 * g + v) * WLD + 16 * t + r] = pk[v];
        }
        *(v4bf *)(sDA2T + (16 * t + r) * SLD + s0 + 4 * g) = pk;
    }
    wave_lds_sync();   // Hs is the wave's own; sDA2T is read after later barriers

    // ---- dL/dh1 = W2^T dL/da2, dL/da1 = dL/dh1 (1 - h1^2), h1 recomputed in FP32
    {
        v8bf Ad[4];
#pragma unroll
        for (int ks = 0; ks < 4; ks++) Ad[ks] = *(const v8bf *)(Hs + r * WLD + 32 * ks + 8 * g);
        v4f dh1[8];
#pragma unroll
        for (int t = 0; t < 8; t++) dh1[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
#pragma unroll
            for (int t = 0; t < 8; t++) dh1[t] = mfma(Ad[ks], B2[8 * ks + t], dh1[t]);
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int k = 16 * t + r;
            float wk[7];
#pragma unroll
            for (int d = 0; d < D; d++) wk[d] = W1[k * D + d];
            const float bk = b1[k];
            v4bf pk;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int s = s0 + 4 * g + v;
                float a = bk;
#pragma unroll
                for (int d = 0; d < D; d++) a = fmaf(wk[d], sZ[s * 8 + d], a);
                const float h = ftanh(a);
                pk[v] = (__bf16)(dh1[t][v] * (1.f - h * h));
            }
            *(v4bf *)(sDA1T + k * SLD + s0 + 4 * g) = pk;
        }
    }
    lacc += __shfl_xor(lacc, 16);
    lacc += __shfl_xor(lacc, 32);
    if (lane == 0) sLoss[w] = lacc;
    __syncthreads();

    // ---- weight gradients over the workgroup's 64 samples
    float *P = part + (size_t)blockIdx.x * NPART;
    // (products taken as (dL/dW)^T tiles, so that each lane holds four
    // consecutive k of one output row: one 16-byte store per lane and tile)
    for (int q = w; q < 21 * 8; q += 4) {
        const int ot = q >> 3, kt = q & 7;
        v4f a = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ks++) {
            const v8bf A = *(const v8bf *)(sDOT + (16 * ot + r) * SLD + 32 * ks + 8 * g);
            const v8bf B = *(const v8bf *)(sH2T + (16 * kt + r) * SLD + 32 * ks + 8 * g);
            a = mfma(B, A, a);
        }
        *(v4f *)(P + OFF_W3 + (16 * ot + r) * H + 16 * kt + 4 * g) = a;
    }
    for (int q = w; q < 8 * 8; q += 4) {
        const int ot = q >> 3, kt = q & 7;
        v4f a = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ks++) {
            const v8bf A = *(const v8bf *)(sDA2T + (16 * ot + r) * SLD + 32 * ks + 8 * g);
            const v8bf B = *(const v8bf *)(sH1T + (16 * kt + r) * SLD + 32 * ks + 8 * g);
            a = mfma(B, A, a);
        }
        *(v4f *)(P + OFF_W2 + (16 * ot + r) * H + 16 * kt + 4 * g) = a;
    }
    for (int o = tid; o < O; o += 256) {
        float acc = 0.f;
        for (int s = 0; s < 64; s++) acc += (float)sDOT[o * SLD + s];
        P[OFF_B3 + o] = acc;
    }
    for (int k = tid; k < H; k += 256) {
        float a2 = 0.f, a1 = 0.f;
        for (int s = 0; s < 64; s++) {
            a2 += (float)sDA2T[k * SLD + s];
            a1 += (float)sDA1T[k * SLD + s];
        }
        P[OFF_B2 + k] = a2;
        P[OFF_B1 + k] = a1;
    }
    for (int e = tid; e < H * D; e += 256) {
        const int k = e / D, d = e % D;
        float acc = 0.f;
        for (int s = 0; s < 64; s++) acc = fmaf((float)sDA1T[k * SLD + s], sZ[s * 8 + d], acc);
        P[OFF_W1 + e] = acc;
    }
    if (tid == 0) {
        P[NPARAM] = sLoss[0] + sLoss[1] + sLoss[2] + sLoss[3];
        float ws = 0.f;
        for (int s = 0; s < 64; s++) ws += sWt[s];
        P[NPARAM + 1] = ws;
    }
}

__device__ inline void write_copies(const ile_mdn_dev &M, int j, float th)
{
    const __bf16 b = (__bf16)th;
    if (j >= OFF_W2 && j < OFF_B2) {
        const int q = j - OFF_W2, o = q / H, k = q % H;
        M.W2b[o * H + k] = b;
        M.W2t[k * H + o] = b;
    } else if (j >= OFF_W3 && j < OFF_B3) {
        const int q = j - OFF_W3, o = q / H, k = q % H;
        M.W3b[o * H + k] = b;
        M.W3t[k * W3T_LD + o] = b;
    }
}

__global__ __launch_bounds__(256) void k_mdn_cast(ile_mdn_dev M)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < NPARAM) write_copies(M, j, M.theta[j]);
}

// Sum the partial rows in a fixed order, mask, normalize by the weight sum;
// then one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 weights
// and refresh the BF16 copies.  A workgroup serves 64 parameters with four
// row slices each (rows s, s+4, s+8, ...), so the read of all rows runs at
// four times the occupancy; the slices combine in slice order.
constexpr int UPD_P = 64;   // parameters per workgroup
__global__ __launch_bounds__(256) void k_mdn_update(ile_mdn_dev M, const float *__restrict__ part,
                                                    int np, float *grad, double *loss, int adam,
                                                    float bc1, float bc2, float lr)
{
    __shared__ float red_g[4][UPD_P], red_w[4][UPD_P];
    const int jj = threadIdx.x & (UPD_P - 1), sl = threadIdx.x / UPD_P;
    const int j = blockIdx.x * UPD_P + jj;
    float ws = 0.f, gs = 0.f;
    if (j < NPARAM) {
        // the loads are independent, so unrolling lets many be in flight
#pragma unroll 8
        for (int t = sl; t < np; t += 4) {
            ws += part[(size_t)t * NPART + NPARAM + 1];
            gs += part[(size_t)t * NPART + j];
        }
    }
    red_g[sl][jj] = gs;
    red_w[sl][jj] = ws;
    __syncthreads();
    if (sl != 0 || j >= NPARAM) return;
    gs = ((red_g[0][jj] + red_g[1][jj]) + red_g[2][jj]) + red_g[3][jj];
    ws = ((red_w[0][jj] + red_w[1][jj]) + red_w[2][jj]) + red_w[3][jj];
    const float gj = (ws > 0.f && ile_mdn_trainable(j)) ? gs / ws : 0.f;
    if (j == 0 && loss) {
        float ls = 0.f;
        for (int t = 0; t < np; t++) ls += part[(size_t)t * NPART + NPARAM];
        *loss = ws > 0.f ? (double)ls / (double)ws : 0.0;
    }
    if (grad) grad[j] = gj;
    if (!adam) return;
    const float m = 0.9f * M.m[j] + 0.1f * gj;
    const float v = 0.999f * M.v[j] + 0.001f * gj * gj;
    M.m[j] = m;
    M.v[j] = v;
    const float th = M.theta[j] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
    M.theta[j] = th;
    write_copies(M, j, th);
}

// ------------------------------------------------- training-set pieces

// Transform fit, multi-block with fixed partitions and fixed-order merges
// (bit-reproducible).  Tempering of the training weights w = exp(beta (ln w
// - max)) over the finite ln w: beta = 1 if the Kish effective size
// (sum w)^2 / sum w^2 reaches max(1, ess_frac * count), else 30 halvings of
// [0, 1] keeping the lower end whose effective size reaches it.  Then the
// weighted circular means of ra, psi, phi (origins) and the weighted mean
// and standard deviation of z = logit(u) (scale >= 1e-3).
//
// Workspace ws: [0, 16) the state below, [16, 16 + FB * 16) block partials.
constexpr int FB = 256;   // blocks of the partial-sum kernels
enum { S_MAX = 0, S_TARGET, S_LO, S_HI, S_BEVAL, S_BETA, S_DONE, S_CNT };

// fixed-order tree sum of `nv` values per thread over a 256-thread block;
// thread 0 writes them to out[0..nv)
template <int NV>
__device__ inline void block_sums256(double (&v)[NV], double *red, double *out)
{
    for (int q = 0; q < NV; q++) {
        red[threadIdx.x] = v[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_fit_max(const double *__restrict__ lnw, int64_t n,
                                                 double *ws)
{
    __shared__ double red[256];
    double mx = -INFINITY, cnt = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)FB * 256)
        if (isfinite(lnw[i])) {
            mx = fmax(mx, lnw[i]);
            cnt += 1.0;
        }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double bm = red[0];
    __syncthreads();
    double c1[1] = {cnt};
    double *P = ws + 16 + blockIdx.x * 16;
    block_sums256<1>(c1, red, P + 1);
    if (threadIdx.x == 0) P[0] = bm;
}

__global__ void k_fit_init(double *ws, double ess_frac)
{
    if (threadIdx.x != 0) return;
    double mx = -INFINITY, cnt = 0.0;
    for (int b = 0; b < FB; b++) {
        mx = fmax(mx, ws[16 + b * 16]);
        cnt += ws[16 + b * 16 + 1];
    }
    ws[S_MAX] = mx;
    ws[S_CNT] = cnt;
    ws[S_TARGET] = fmax(1.0, ess_frac * cnt);
    ws[S_LO] = 0.0;
    ws[S_HI] = 1.0;
    ws[S_BEVAL] = 1.0;
    ws[S_BETA] = 1.0;
    ws[S_DONE] = cnt > 0 ? 0.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_fit_ess_part(const double *__restrict__ lnw, int64_t n,
                                                      double *ws)
{
    __shared__ double red[256];
    if (ws[S_DONE] != 0.0) return;   // uniform across the grid
    const double m = ws[S_MAX], beta = ws[S_BEVAL];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)FB * 256) {
        if (!isfinite(lnw[i])) continue;
        const double e = exp(beta * (lnw[i] - m));
        v[0] += e;
        v[1] += e * e;
    }
    block_sums256<2>(v, red, ws + 16 + blockIdx.x * 16);
}

// it = 0 judges beta = 1; it = 1..30 halve [lo, hi]
__global__ void k_fit_ess_step(double *ws, int it)
{
    if (threadIdx.x != 0 || ws[S_DONE] != 0.0) return;
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < FB; b++) {
        s1 += ws[16 + b * 16];
        s2 += ws[16 + b * 16 + 1];
    }
    const bool ok = s2 > 0.0 && s1 * s1 / s2 >= ws[S_TARGET];
    if (it == 0) {
        if (ok) {
            ws[S_BETA] = 1.0;
            ws[S_DONE] = 1.0;
            return;
        }
    } else if (ok) {
        ws[S_LO] = ws[S_BEVAL];
    } else {
        ws[S_HI] = ws[S_BEVAL];
    }
    ws[S_BETA] = ws[S_LO];
    ws[S_BEVAL] = 0.5 * (ws[S_LO] + ws[S_HI]);
}

__device__ inline double fit_weight(const double *ws, double l)
{
    return isfinite(l) ? exp(ws[S_BETA] * (l - ws[S_MAX])) : 0.0;
}

__global__ __launch_bounds__(256) void k_fit_circ_part(const double *__restrict__ x, int64_t ld,
                                                       const double *__restrict__ lnw, int64_t n,
                                                       double *ws)
{
    __shared__ double red[256];
    const int pd[3] = {0, 2, 3};
    const double per[3] = {kTwoPi, kPi, kTwoPi};
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)FB * 256) {
        const double wi = fit_weight(ws, lnw[i]);
        if (wi == 0.0) continue;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double sn, cs;
            sincos(kTwoPi * x[pd[j] * ld + i] / per[j], &sn, &cs);
            v[2 * j] += wi * cs;
            v[2 * j + 1] += wi * sn;
        }
    }
    block_sums256<6>(v, red, ws + 16 + blockIdx.x * 16);
}

__global__ void k_fit_circ_fin(double *ws, ile_mdn_tr *tr)
{
    if (threadIdx.x != 0) return;
    const double per[3] = {kTwoPi, kPi, kTwoPi};
    for (int j = 0; j < 3; j++) {
        double sc = 0.0, ss = 0.0;
        for (int b = 0; b < FB; b++) {
            sc += ws[16 + b * 16 + 2 * j];
            ss += ws[16 + b * 16 + 2 * j + 1];
        }
        tr->origin[j] = atan2(ss, sc) * per[j] / kTwoPi;
    }
}

__global__ __launch_bounds__(256) void k_fit_mom_part(const double *__restrict__ x, int64_t ld,
                                                      const double *__restrict__ lnw, int64_t n,
                                                      const ile_mdn_tr *__restrict__ trp, double *ws)
{
    __shared__ double red[256];
    const ile_mdn_tr T = *trp;
    double v[15];
    for (int q = 0; q < 15; q++) v[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)FB * 256) {
        const double wi = fit_weight(ws, lnw[i]);
        if (wi == 0.0) continue;
        double zz[7];
        bool ok = true;
        for (int d = 0; d < D; d++) {
            double ldu;
            const double u = to_unit(T, d, x[d * ld + i], ldu);
            if (!(u > 0.0 && u < 1.0)) ok = false;
            else zz[d] = log(u) - log1p(-u);
        }
        if (!ok) continue;
        v[0] += wi;
        for (int d = 0; d < D; d++) {
            v[1 + d] += wi * zz[d];
            v[8 + d] += wi * zz[d] * zz[d];
        }
    }
    block_sums256<15>(v, red, ws + 16 + blockIdx.x * 16);
}

__global__ void k_fit_stats_only(const double *ws, double *stats)
{
    if (threadIdx.x != 0) return;
    stats[0] = ws[S_MAX];
    stats[1] = ws[S_BETA];
}

__global__ void k_fit_mom_fin(double *ws, ile_mdn_tr *tr, double *stats)
{
    if (threadIdx.x != 0) return;
    double v[15];
    for (int q = 0; q < 15; q++) {
        v[q] = 0.0;
        for (int b = 0; b < FB; b++) v[q] += ws[16 + b * 16 + q];
    }
    for (int d = 0; d < D; d++) {
        const double m = v[0] > 0 ? v[1 + d] / v[0] : 0.0;
        const double var = v[0] > 0 ? v[8 + d] / v[0] - m * m : 1.0;
        tr->mean[d] = m;
        tr->scale[d] = fmax(sqrt(fmax(var, 0.0)), 1e-3);
    }
    stats[0] = ws[S_MAX];
    stats[1] = ws[S_BETA];
}

// z~ (FP32, [7][n]) and training weights: tempered exp(beta (ln w - max))
// when lnw is given, else w_in (or 1); 0 where the transform is undefined.
__global__ __launch_bounds__(256) void k_mdn_prepare(const ile_mdn_tr *__restrict__ trp,
                                                     const double *__restrict__ x, int64_t ld,
                                                     const double *__restrict__ lnw,
                                                     const double *__restrict__ w_in, int64_t n,
                                                     const double *__restrict__ stats, float *z,
                                                     double *w)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const ile_mdn_tr T = *trp;
    double xi[7];
    for (int d = 0; d < D; d++) xi[d] = x[d * ld + i];
    float zz[7];
    const double lj = to_z(T, xi, zz);
    for (int d = 0; d < D; d++) z[d * n + i] = zz[d];
    double wi = w_in ? w_in[i] : 1.0;
    if (lnw) wi = isfinite(lnw[i]) ? exp(stats[1] * (lnw[i] - stats[0])) : 0.0;
    w[i] = lj == -INFINITY ? 0.0 : wi;
}

// inclusive prefix sums: CB blocks of 256 threads, each thread a contiguous
// chunk; chunk totals are scanned in order by one thread, then each chunk
// is written from its offset (fixed order: bit-reproducible)
constexpr int CB = 64;
__global__ __launch_bounds__(256) void k_mdn_cdf_part(const double *__restrict__ w, int64_t n,
                                                      double *tot)
{
    const int64_t T = (int64_t)CB * 256, per = (n + T - 1) / T;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t lo = t * per < n ? t * per : n, hi = lo + per < n ? lo + per : n;
    double s = 0.0;
    for (int64_t i = lo; i < hi; i++) s += w[i];
    tot[t] = s;
}

// exclusive scan of the CB * 256 chunk totals: each of 256 threads scans 64
// consecutive totals, thread 0 scans the 256 thread sums, each thread adds
// its offset (fixed order)
__global__ __launch_bounds__(256) void k_mdn_cdf_scan(double *tot)
{
    __shared__ double ts[256];
    constexpr int PER = CB;   // CB * 256 totals over 256 threads
    double *mine = tot + (size_t)threadIdx.x * PER;
    double run = 0.0;
    for (int i = 0; i < PER; i++) {
        const double v = mine[i];
        mine[i] = run;
        run += v;
    }
    ts[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int t = 0; t < 256; t++) {
            const double v = ts[t];
            ts[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    const double off = ts[threadIdx.x];
    for (int i = 0; i < PER; i++) mine[i] += off;
}

__global__ __launch_bounds__(256) void k_mdn_cdf_write(const double *__restrict__ w, int64_t n,
                                                       const double *__restrict__ tot, double *cdf)
{
    const int64_t T = (int64_t)CB * 256, per = (n + T - 1) / T;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t lo = t * per < n ? t * per : n, hi = lo + per < n ? lo + per : n;
    double run = tot[t];
    for (int64_t i = lo; i < hi; i++) {
        run += w[i];
        cdf[i] = run;
    }
}

// draw b of a training call: training index drawn with probability
// w_i / sum w (independent draws; step t of the call uses draws
// t*batch .. t*batch + batch - 1)
__global__ __launch_bounds__(256) void k_mdn_draw_idx(uint64_t seed, int64_t count,
                                                      const double *__restrict__ cdf, int64_t n,
                                                      int32_t *idx)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= count) return;
    uint32_t q[4];
    ile_rng::block(seed, (uint64_t)b, 0u, ile_rng::kTagTrain, q);
    const double target = ile_rng::u53(q[0], q[1]) * cdf[n - 1];
    int64_t lo = 0, hi = n - 1;   // first i with cdf[i] > target
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    idx[b] = (int32_t)lo;
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t ile_launch_mdn_cast(const ile_mdn_dev &M, hipStream_t st)
{
    hipLaunchKernelGGL(k_mdn_cast, dim3((NPARAM + 255) / 256), dim3(256), 0, st, M);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_logpdf(const ile_mdn_dev &M, const ile_mdn_mix &mix, const double *x,
                                 int64_t ld, int64_t n, double *ln_q, int grid, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (mix.nb > MAXB) return hipErrorInvalidValue;
    const int64_t tiles = (n + 63) / 64;
    grid = (int)std::min<int64_t>(tiles, std::max(grid, 1));
    hipLaunchKernelGGL(k_mdn_infer<false>, dim3(grid), dim3(256), 0, st, M.theta, M.W2b, M.W3b,
                       M.tr, mix, (uint64_t)0, (int64_t)0, n, const_cast<double *>(x), ld,
                       (double *)nullptr, ln_q);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_sample(const ile_mdn_dev &M, const ile_mdn_mix &mix, uint64_t seed,
                                 int64_t first, int64_t n, double *x, int64_t ld, double *ln_p,
                                 double *ln_q, int grid, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (mix.nb > MAXB) return hipErrorInvalidValue;
    const int64_t tiles = (n + 63) / 64;
    grid = (int)std::min<int64_t>(tiles, std::max(grid, 1));
    hipLaunchKernelGGL(k_mdn_infer<true>, dim3(grid), dim3(256), 0, st, M.theta, M.W2b, M.W3b,
                       M.tr, mix, seed, first, n, x, ld, ln_p, ln_q);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_fit(const double *x, int64_t ld, const double *lnw, int64_t n,
                              double ess_frac, ile_mdn_tr *tr, double *stats, double *ws,
                              bool fit_transform, hipStream_t st)
{
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fit_max, dim3(FB), dim3(256), 0, st, lnw, n, ws);
    hipLaunchKernelGGL(k_fit_init, dim3(1), dim3(64), 0, st, ws, ess_frac);
    for (int it = 0; it <= 30; it++) {
        hipLaunchKernelGGL(k_fit_ess_part, dim3(FB), dim3(256), 0, st, lnw, n, ws);
        hipLaunchKernelGGL(k_fit_ess_step, dim3(1), dim3(64), 0, st, ws, it);
    }
    if (fit_transform) {
        hipLaunchKernelGGL(k_fit_circ_part, dim3(FB), dim3(256), 0, st, x, ld, lnw, n, ws);
        hipLaunchKernelGGL(k_fit_circ_fin, dim3(1), dim3(64), 0, st, ws, tr);
        hipLaunchKernelGGL(k_fit_mom_part, dim3(FB), dim3(256), 0, st, x, ld, lnw, n,
                           (const ile_mdn_tr *)tr, ws);
        hipLaunchKernelGGL(k_fit_mom_fin, dim3(1), dim3(64), 0, st, ws, tr, stats);
    } else {
        hipLaunchKernelGGL(k_fit_stats_only, dim3(1), dim3(64), 0, st, ws, stats);
    }
    return hipGetLastError();
}

size_t ile_mdn_fit_ws_doubles() { return std::max<size_t>(16 + (size_t)FB * 16, (size_t)CB * 256); }

hipError_t ile_launch_mdn_prepare(const ile_mdn_tr *tr, const double *x, int64_t ld,
                                  const double *lnw, int64_t n, const double *stats, float *z,
                                  double *w, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdn_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tr,
                       x, ld, lnw, (const double *)nullptr, n, stats, z, w);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_prepare_w(const ile_mdn_tr *tr, const double *x, int64_t ld,
                                    const double *w_in, int64_t n, float *z, double *w,
                                    hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdn_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tr,
                       x, ld, (const double *)nullptr, w_in, n, (const double *)nullptr, z, w);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_cdf(const double *w, int64_t n, double *cdf, double *ws,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdn_cdf_part, dim3(CB), dim3(256), 0, st, w, n, ws);
    hipLaunchKernelGGL(k_mdn_cdf_scan, dim3(1), dim3(256), 0, st, ws);
    hipLaunchKernelGGL(k_mdn_cdf_write, dim3(CB), dim3(256), 0, st, w, n, (const double *)ws, cdf);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_draw_idx(uint64_t seed, int64_t count, const double *cdf, int64_t n,
                                   int32_t *idx, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdn_draw_idx, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       seed, count, cdf, n, idx);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_grad(const ile_mdn_dev &M, const float *z, int64_t ldz,
                               const int32_t *idx, const double *w, int batch, float *part,
                               hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdn_grad, dim3((batch + 63) / 64), dim3(256), 0, st, M.theta, M.W2b,
                       M.W3b, M.W2t, M.W3t, M.tr, z, ldz, idx, w, batch, part);
    return hipGetLastError();
}

hipError_t ile_launch_mdn_update(const ile_mdn_dev &M, const float *part, int n_part,
                                 float *grad, double *loss, bool adam, int64_t step, double lr,
                                 hipStream_t st)
{
    const double s = (double)std::max<int64_t>(step, 1);
    const float bc1 = (float)(1.0 - pow(0.9, s)), bc2 = (float)(1.0 - pow(0.999, s));
    hipLaunchKernelGGL(k_mdn_update, dim3((NPARAM + UPD_P - 1) / UPD_P), dim3(256), 0, st, M, part,
                       n_part, grad, loss, adam ? 1 : 0, bc1, bc2, (float)lr);
    return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void k_lnw(const double *__restrict__ lnL,
                                             const double *__restrict__ lp,
                                             const double *__restrict__ lq, int64_t n,
                                             double *lnw)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) lnw[i] = lnL[i] + (lp ? lp[i] : 0.0) - (lq ? lq[i] : 0.0);
}
}  // namespace

hipError_t ile_launch_lnw(const double *lnL, const double *ln_p, const double *ln_q, int64_t n,
                          double *lnw, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lnw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lnL, ln_p,
                       ln_q, n, lnw);
    return hipGetLastError();
}
