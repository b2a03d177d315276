"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module; the product package never does.  The arithmetic lives in
ile_oracle.c (plain C, FP64, no FMA contraction); the numpy code here builds
the physically consistent injection instance and the direct form of the
likelihood used to pin it, both written from the paper:

* Eq. (1): ln L = sum_k <h_k|d_k> - <h_k|h_k>/2 (the printed bracket of
  Eq. (1) is misplaced; this is the reading consistent with Eq. (7));
* Eq. (2) with a white noise spectrum: <a|b> = sum_i conj(a_i) b_i;
* Eq. (8): Q_k,lm(s) = <h_lm shifted by s | d_k>, U = <h_lm|h_l'm'>,
  V = <h_lm^*|h_l'm'>.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libile_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


class OrcConfig(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("n_lm", C.c_int32),
                ("modes", C.POINTER(C.c_int32)), ("srate_hz", C.c_double),
                ("n_t", C.c_int32), ("d_ref_mpc", C.c_double),
                ("gmst_rad", C.c_double), ("earth_radius_m", C.c_double),
                ("t0_s", C.c_double), ("n_q", C.c_int64)]


class OrcDetector(C.Structure):
    _fields_ = [("lat_deg", C.c_double), ("lon_deg", C.c_double),
                ("xarm_az_deg", C.c_double)]


class OrcResult(C.Structure):
    _fields_ = [("ln_L_marg", C.c_double), ("n_eff", C.c_double),
                ("n_eff_kish", C.c_double), ("sigma", C.c_double),
                ("max_lnL", C.c_double), ("n_samples", C.c_int64)]


def lib():
    """Load the oracle library: ILE_ORACLE_LIB names another build of it
    (the sanitizer build), else oracle/libile_oracle.so, built if missing."""
    global _lib
    if _lib is None:
        path = os.environ.get("ILE_ORACLE_LIB") or _LIB_PATH
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = C.CDLL(path)
        _lib.orc_delay.restype = C.c_double
        _lib.orc_logmeanexp.restype = C.c_double
        _lib.orc_eval.restype = C.c_int64
        _lib.orc_lnL_series.restype = C.c_int
        _lib.orc_lnL_series_at.restype = C.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


# ------------------------------------------------------------- geometry
def detector_frame(det, R=6378.0e3):
    r = np.zeros(3)
    D = np.zeros(9)
    d = OrcDetector(*det)
    lib().orc_detector_frame(C.byref(d), C.c_double(R), _p(r), _p(D))
    return r, D.reshape(3, 3)


def antenna(D, ra, dec, psi, gmst=0.0):
    D = np.ascontiguousarray(D, np.float64).reshape(9)
    fp, fx = C.c_double(), C.c_double()
    lib().orc_antenna(_p(D), C.c_double(ra), C.c_double(dec), C.c_double(psi),
                      C.c_double(gmst), C.byref(fp), C.byref(fx))
    return fp.value, fx.value


def delay(r, ra, dec, gmst=0.0):
    r = np.ascontiguousarray(r, np.float64)
    return lib().orc_delay(_p(r), C.c_double(ra), C.c_double(dec),
                           C.c_double(gmst))


def sylm(l, m, theta, phi):
    re, im = C.c_double(), C.c_double()
    lib().orc_sylm(int(l), int(m), C.c_double(theta), C.c_double(phi),
                   C.byref(re), C.byref(im))
    return complex(re.value, im.value)


# ------------------------------------------------------------ likelihood
class Ctx:
    """Holds one instance in the oracle's C structures."""

    def __init__(self, inst):
        self.inst = inst
        self.modes = np.ascontiguousarray(np.array(inst.modes, np.int32).reshape(-1))
        self.cfg = OrcConfig(inst.n_det, inst.n_lm,
                             self.modes.ctypes.data_as(C.POINTER(C.c_int32)),
                             inst.srate_hz, inst.n_t, inst.d_ref_mpc,
                             inst.gmst_rad, inst.earth_radius_m, inst.t0_s,
                             inst.n_q)
        self.dets = (OrcDetector * inst.n_det)(*[OrcDetector(*d) for d in inst.dets])
        self.Q = np.ascontiguousarray(inst.Q, np.complex128).view(np.float64)
        self.U = np.ascontiguousarray(inst.U, np.complex128).view(np.float64)
        self.V = np.ascontiguousarray(inst.V, np.complex128).view(np.float64)

    def window_position(self, theta):
        th = np.ascontiguousarray(theta, np.float64)
        x = np.zeros(self.inst.n_det)
        lib().orc_window_position(C.byref(self.cfg), self.dets, _p(th), _p(x))
        return x

    def lnL_series(self, theta, s_start=None):
        th = np.ascontiguousarray(theta, np.float64)
        out = np.zeros(self.inst.n_t)
        if s_start is None:
            rc = lib().orc_lnL_series(C.byref(self.cfg), _p(self.Q), _p(self.U),
                                      _p(self.V), self.dets, _p(th), _p(out))
        else:
            s = np.ascontiguousarray(s_start, np.int64)
            rc = lib().orc_lnL_series_at(C.byref(self.cfg), _p(self.Q),
                                         _p(self.U), _p(self.V), self.dets,
                                         _p(th), s.ctypes.data_as(_i64p), _p(out))
        if rc != 0:
            raise ValueError("window outside Q or invalid sample")
        return out

    def eval(self, samples, n_threads=0):
        s = np.ascontiguousarray(samples, np.float64)
        n = s.shape[1]
        out = np.zeros(n)
        lib().orc_eval(C.byref(self.cfg), _p(self.Q), _p(self.U), _p(self.V),
                       self.dets, _p(s), C.c_int64(n), _p(out), int(n_threads))
        return out


def logmeanexp(x):
    x = np.ascontiguousarray(x, np.float64)
    return lib().orc_logmeanexp(_p(x), C.c_int64(x.size))


def integrate(lnLmargT, ln_p, ln_q):
    a = np.ascontiguousarray(lnLmargT, np.float64)
    b = np.ascontiguousarray(ln_p, np.float64)
    c = np.ascontiguousarray(ln_q, np.float64)
    r = OrcResult()
    lib().orc_integrate(_p(a), _p(b), _p(c), C.c_int64(a.size), C.byref(r))
    return dict(ln_L_marg=r.ln_L_marg, n_eff=r.n_eff, n_eff_kish=r.n_eff_kish,
                sigma=r.sigma, max_lnL=r.max_lnL, n_samples=r.n_samples)


# ------------------------------------------ Q, U, V from the frequency domain
def fft_freqs(n_q, df):
    """Frequencies of the n_q-point FFT grid: i df for i < n_q/2, else
    (i - n_q) df."""
    i = np.arange(n_q)
    return np.where(i < n_q // 2, i, i - n_q) * df


def qvu_fd(h_f, d_f, psd, df, f_min, f_max, t0, s_idx=None):
    """Q, U, V of Eq. (8) from frequency-domain series, each inner product
    the band-limited noise-weighted integral of Eq. (2) taken as a sum over
    the FFT grid f_i with spacing df:
        <a|b>_k = 2 df sum_{f_min < |f_i| < f_max} conj(a_i) b_i / S_k,i,
        Q_k,lm(t) = 2 df sum_i exp(2 pi i f_i t) conj(h_lm,i) d_k,i / S_k,i,
        U_k = <h_lm|h_l'm'>_k,  V_k = <h*_lm|h_l'm'>_k,
    where the transform of conj(h) at f is conj(h(-f)), so V's summand is
    h_lm(-f_i) h_l'm'(f_i) / S_k,i.  h_f [n_lm][n], d_f [n_det][n] complex,
    psd [n_det][n] the spectrum at |f_i|.  Q at the times t0 + s/(n df) for
    s in s_idx (default all n), as the direct sum (no FFT)."""
    h_f = np.asarray(h_f, np.complex128)
    d_f = np.asarray(d_f, np.complex128)
    psd = np.asarray(psd, np.float64)
    n = h_f.shape[1]
    f = fft_freqs(n, df)
    band = (np.abs(f) > f_min) & (np.abs(f) < f_max)
    w = np.where(band[None, :], 2.0 * df / np.where(band[None, :], psd, 1.0), 0.0)
    s_idx = np.arange(n) if s_idx is None else np.asarray(s_idx)
    t = t0 + s_idx / (n * df)
    E = np.exp(2j * np.pi * np.outer(f, t))            # [n][len(s)]
    n_det, n_lm = d_f.shape[0], h_f.shape[0]
    Q = np.zeros((n_det, n_lm, s_idx.size), np.complex128)
    for k in range(n_det):
        for a in range(n_lm):
            Q[k, a] = (w[k] * np.conj(h_f[a]) * d_f[k]) @ E
    neg = (-np.arange(n)) % n                           # index of -f_i
    U = np.zeros((n_det, n_lm, n_lm), np.complex128)
    V = np.zeros((n_det, n_lm, n_lm), np.complex128)
    for k in range(n_det):
        for a in range(n_lm):
            for b in range(n_lm):
                U[k, a, b] = np.sum(w[k] * np.conj(h_f[a]) * h_f[b])
                V[k, a, b] = np.sum(w[k] * h_f[a][neg] * h_f[b])
    return Q, U, V


# ------------------------------------------- surrogate (reduced-order) form
def rom_coeffs(A, lam):
    """Surrogate coefficients c_lm,b(lambda) = sum_p A[lm][b][p] lambda^p of
    the linear representation h_lm(lambda; t) = sum_b c_lm,b(lambda) e_b(t)
    (Sec. V: a linear basis for h_lm enabling likelihoods as a function of
    both extrinsic and intrinsic parameters).  A complex [n_lm][n_b][P]."""
    A = np.asarray(A, np.complex128)
    return np.tensordot(A, lam ** np.arange(A.shape[2]), axes=([2], [0]))


def rom_instance(basis, modes, A, lam):
    """The Eq. (8) quantities at lambda from the basis overlaps held in
    `basis` (Q^B_k,b(t) = <e_b(t)|d>_k, G_k = <e_b|e_b'>_k, H_k =
    <e_b*|e_b'>_k as its Q, U, V), by linearity of Eq. (2):
        Q_k,lm(t) = sum_b conj(c_lm,b) Q^B_k,b(t),
        U_k = conj(C) G_k C^T,   V_k = C H_k C^T   (C = [c_lm,b])."""
    import copy
    C = rom_coeffs(A, lam)
    inst = copy.copy(basis)
    inst.modes = list(modes)
    inst.Q = np.einsum("ab,kbs->kas", np.conj(C), basis.Q)
    inst.U = np.stack([np.conj(C) @ basis.U[k] @ C.T for k in range(basis.n_det)])
    inst.V = np.stack([C @ basis.V[k] @ C.T for k in range(basis.n_det)])
    return inst


def rom_eval(basis, modes, A, samples8):
    """ln L_margT of joint samples [8][N] (7 extrinsic rows, then lambda) by
    the definition: the surrogate's Q, U, V at each sample's lambda, then
    Eq. (7) and Eq. (9) as in Ctx.eval."""
    s = np.asarray(samples8, np.float64)
    out = np.empty(s.shape[1])
    for i in range(s.shape[1]):
        inst = rom_instance(basis, modes, A, s[7, i])
        out[i] = Ctx(inst).eval(s[:7, i:i + 1])[0]
    return out


# ------------------------------------------------ extrinsic harvest
def inverse_cdf(c, target):
    """Inverse-CDF pick on inclusive cumulative weights c: the first index
    i with c[i] > target; when rounding leaves target at or above the total,
    the first index whose cumulative weight reaches the total (so an index
    of zero weight is never returned)."""
    i = int(np.searchsorted(c, target, side="right"))
    if i >= c.size:
        i = int(np.searchsorted(c, c[-1], side="left"))
    return i


def harvest(ctx, samples, ln_p, ln_q, u):
    """Joint extrinsic posterior draws from one final Monte Carlo iteration
    (Sec. V: joint intrinsic and extrinsic information harvested from a
    single final iteration; Eq. (3) at fixed intrinsic parameters).

    The draws theta_alpha with log prior ln_p and log proposal ln_q, and the
    bin grid t_j of Eq. (9), carry the joint weight
        P(alpha, j)  proportional to  exp(ln p_alpha - ln q_alpha + L_alpha,j),
    which factors into a sample draw with weight exp(lnLmargT + ln p - ln q)
    (Eq. (4)'s weight) and a bin draw with weight exp(L_alpha,j) given the
    sample.  Draw k takes the sample by inverse CDF of uniform u[0][k] on
    the cumulative sample weights (index order), then the bin by inverse CDF
    of u[1][k] on that sample's cumulative bin weights.  Bin j means the
    geocentre time t_ref + (j - (n_t-1)/2)/srate.

    Returns (idx [n_out] int64, bin [n_out] int32, theta [7][n_out]) with
    theta the chosen sample with row 6 replaced by the bin time."""
    inst = ctx.inst
    s = np.ascontiguousarray(samples, np.float64)
    u = np.asarray(u, np.float64).reshape(2, -1)
    lnL = ctx.eval(s)
    if not np.all(np.isfinite(lnL)):
        raise ValueError("invalid sample")
    lw = lnL + np.asarray(ln_p, np.float64) - np.asarray(ln_q, np.float64)
    lw = np.where(np.isfinite(lw), lw, -np.inf)
    if not np.any(np.isfinite(lw)):
        raise ValueError("no sample with positive weight")
    c = np.cumsum(np.exp(lw - lw.max()))
    n_out = u.shape[1]
    idx = np.zeros(n_out, np.int64)
    bins = np.zeros(n_out, np.int32)
    theta = np.zeros((7, n_out))
    h = (inst.n_t - 1) // 2
    for k in range(n_out):
        a = inverse_cdf(c, u[0, k] * c[-1])
        L = ctx.lnL_series(s[:, a])
        cj = np.cumsum(np.exp(L - L.max()))
        j = inverse_cdf(cj, u[1, k] * cj[-1])
        idx[k], bins[k] = a, j
        theta[:, k] = s[:, a]
        theta[6, k] = s[6, a] + (j - h) / inst.srate_hz
    return idx, bins, theta


# ------------------------------------------------------------ sampling
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def prior_draw(seed, first, n, d_min=10.0, d_max=1000.0, t_ref_max=0.01):
    s = np.zeros((7, n))
    lp = np.zeros(n)
    lib().orc_prior_draw(C.c_uint64(seed), C.c_int64(first), C.c_int64(n),
                         C.c_double(d_min), C.c_double(d_max),
                         C.c_double(t_ref_max), _p(s), C.c_int64(n), _p(lp))
    return s, lp


def hist_draw(seed, first, n, P_ra, P_sd, d_min=10.0, d_max=1000.0, t_ref_max=0.01):
    """Draws from the histogram proposal (ra, sin dec) x prior; returns
    samples [7][n], ln p, ln q and the bins [2][n]."""
    P_ra = np.ascontiguousarray(P_ra, np.float64)
    P_sd = np.ascontiguousarray(P_sd, np.float64)
    nb = P_ra.size
    s = np.zeros((7, n))
    lp = np.zeros(n)
    lq = np.zeros(n)
    bins = np.zeros((2, n), np.int32)
    lib().orc_hist_draw(C.c_uint64(seed), C.c_int64(first), C.c_int64(n), int(nb),
                        _p(P_ra), _p(P_sd), C.c_double(d_min), C.c_double(d_max),
                        C.c_double(t_ref_max), _p(s), C.c_int64(n), _p(lp), _p(lq),
                        bins.ctypes.data_as(C.POINTER(C.c_int32)))
    return s, lp, lq, bins


def hist_refit(bins, lnw, nb, floor=0.1, scale=10.0):
    bins = np.ascontiguousarray(bins, np.int32)
    lnw = np.ascontiguousarray(lnw, np.float64)
    n = lnw.size
    P_ra = np.zeros(nb)
    P_sd = np.zeros(nb)
    lib().orc_hist_refit(bins.ctypes.data_as(C.POINTER(C.c_int32)), C.c_int64(n),
                         _p(lnw), C.c_int64(n), int(nb), C.c_double(floor),
                         C.c_double(scale), _p(P_ra), _p(P_sd))
    return P_ra, P_sd


# ------------------------------------------------- injection (pins only)
def mode_factors(inst, theta):
    """(F_k = F+ + i Fx per detector, -2Y_lm(iota, phi) per mode)."""
    F = np.zeros(inst.n_det, np.complex128)
    for k, d in enumerate(inst.dets):
        _, D = detector_frame(d, inst.earth_radius_m)
        fp, fx = antenna(D, theta[0], theta[1], theta[2], inst.gmst_rad)
        F[k] = fp + 1j * fx
    iota = np.arccos(theta[4])
    Y = np.array([sylm(l, m, iota, theta[3]) for (l, m) in inst.modes])
    return F, Y


def detector_response(inst, h_lm, theta, lag):
    """h_k[i] = Re(F_k (Dref/D) sum_lm Y_lm h_lm[i - lag_k]) (Eqs. (5), (6)
    and the detector response below Eq. (6), white-noise discrete form with
    circular shifts)."""
    F, Y = mode_factors(inst, theta)
    kappa = inst.d_ref_mpc / theta[5]
    out = np.zeros((inst.n_det, h_lm.shape[1]))
    for k in range(inst.n_det):
        z = np.zeros(h_lm.shape[1], np.complex128)
        for a in range(inst.n_lm):
            z += Y[a] * np.roll(h_lm[a], int(lag[k]))
        out[k] = (F[k] * kappa * z).real
    return out


def inner(a, b):
    """Eq. (2) for white noise, discrete: sum_i conj(a_i) b_i."""
    return np.vdot(a, b)


def direct_lnL(data, model):
    """Eq. (1) as read: sum_k -1/2 (<h_k - d_k|h_k - d_k> - <d_k|d_k>)."""
    tot = 0.0
    for k in range(data.shape[0]):
        r = model[k] - data[k]
        tot += -0.5 * (inner(r, r).real - inner(data[k], data[k]).real)
    return tot


def injection_instance(base, h_lm, theta_inj, noise_sigma=0.0, rng=None, snr=None):
    """Physically consistent instance: the data d_k is the response to
    theta_inj (zero noise unless noise_sigma > 0), and Q, U, V are the
    white-noise inner products of Eq. (8) with circular shifts.

    Q index s of the instance corresponds to arrival lag s - n_q/2 samples
    after the start of h_lm, matching t0 = -(n_q/2) dt.  With snr, the
    (noise-free) data are scaled to network SNR sqrt(sum_k <d_k|d_k>) = snr,
    i.e. the injected distance becomes theta_inj[5] / scale
    (inst.meta["d_inj"]).
    Returns (instance, data, injected lags)."""
    import copy
    inst = copy.copy(base)
    n = h_lm.shape[1]
    dt = 1.0 / inst.srate_hz
    t0 = -(n // 2) * dt
    lags = []
    for k, d in enumerate(inst.dets):
        r, _ = detector_frame(d, inst.earth_radius_m)
        tau = delay(r, theta_inj[0], theta_inj[1], inst.gmst_rad)
        x = (theta_inj[6] + tau - t0) / dt
        lags.append(int(np.floor(x + 0.5)))
    lags = np.array(lags)
    data = detector_response(inst, h_lm, theta_inj, lags)
    scale = 1.0
    if snr is not None and snr > 0:
        scale = snr / math.sqrt(sum(float(np.dot(d, d)) for d in data))
        data = data * scale
    if noise_sigma > 0:
        data = data + noise_sigma * rng.standard_normal(data.shape)
    A = h_lm.T  # [i, lm]
    U = np.stack([A.conj().T @ A for _ in range(inst.n_det)])
    V = np.stack([A.T @ A for _ in range(inst.n_det)])
    Q = np.zeros((inst.n_det, inst.n_lm, n), np.complex128)
    for k in range(inst.n_det):
        D = np.fft.fft(data[k])
        for a in range(inst.n_lm):
            # Q[s] = sum_i conj(h[(i - s) mod n]) d[i]: circular correlation
            Q[k, a] = np.fft.ifft(np.conj(np.fft.fft(h_lm[a])) * D)
    inst.Q, inst.U, inst.V = Q, U, V
    inst.meta = dict(inst.meta, d_inj=theta_inj[5] / scale, rho2=float(sum(np.dot(d, d) for d in data)))
    return inst, data, lags


# ------------------------------------------------- learned proposal (MDN)
MDN_NPARAM = 60880


class MdnTransform(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("mean", C.c_double * 7),
                ("scale", C.c_double * 7), ("d_min", C.c_double),
                ("d_max", C.c_double), ("t_ref_max", C.c_double),
                ("sigma_floor", C.c_double), ("sigma_scale", C.c_double)]


def mdn_transform(origin=(0.0, 0.0, 0.0), mean=None, scale=None, d_min=10.0,
                  d_max=1000.0, t_ref_max=0.01, sigma_floor=1e-3, sigma_scale=1.0):
    tr = MdnTransform()
    for j in range(3):
        tr.origin[j] = origin[j]
    for d in range(7):
        tr.mean[d] = 0.0 if mean is None else mean[d]
        tr.scale[d] = 1.0 if scale is None else scale[d]
    tr.d_min, tr.d_max, tr.t_ref_max = d_min, d_max, t_ref_max
    tr.sigma_floor = sigma_floor
    tr.sigma_scale = sigma_scale
    return tr


def mdn_mask():
    L = lib()
    return np.array([L.orc_mdn_mask(C.c_int64(j)) for j in range(MDN_NPARAM)], np.int32)


def mdn_to_z(tr, x):
    L = lib()
    L.orc_mdn_to_z.restype = C.c_double
    x = np.ascontiguousarray(x, np.float64)
    z = np.zeros(7)
    lj = L.orc_mdn_to_z(C.byref(tr), _p(x), _p(z))
    return z, lj


def mdn_lnq_z(params, tr, z):
    """(ln q(z~), per-dimension terms)."""
    L = lib()
    L.orc_mdn_lnq_z.restype = C.c_double
    P = np.ascontiguousarray(params, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    dims = np.zeros(7)
    v = L.orc_mdn_lnq_z(_p(P), C.byref(tr), _p(z), _p(dims))
    return v, dims


def mdn_logpdf(params, tr, x):
    P = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[1]
    out = np.zeros(n)
    lib().orc_mdn_logpdf(_p(P), C.byref(tr), _p(x), C.c_int64(n), C.c_int64(n), _p(out))
    return out


def mdn_loss_grad(params, tr, x, w=None):
    P = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[1]
    g = np.zeros(MDN_NPARAM)
    loss = C.c_double()
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, np.float64)
        wp = _p(w)
    lib().orc_mdn_loss_grad(_p(P), C.byref(tr), _p(x), C.c_int64(n), C.c_int64(n), wp,
                            C.byref(loss), _p(g))
    return loss.value, g


def mdn_tempering(lnw, ess_frac=0.01):
    L = lib()
    L.orc_mdn_tempering.restype = C.c_double
    lnw = np.ascontiguousarray(lnw, np.float64)
    m = C.c_double()
    b = L.orc_mdn_tempering(_p(lnw), C.c_int64(lnw.size), C.c_double(ess_frac), C.byref(m))
    return b, m.value


def mdn_fit_transform(x, lnw, ess_frac=0.01, d_min=10.0, d_max=1000.0, t_ref_max=0.01,
                      sigma_floor=1e-3):
    x = np.ascontiguousarray(x, np.float64)
    lnw = np.ascontiguousarray(lnw, np.float64)
    n = x.shape[1]
    tr = mdn_transform(d_min=d_min, d_max=d_max, t_ref_max=t_ref_max,
                       sigma_floor=sigma_floor)
    lib().orc_mdn_fit_transform(_p(x), C.c_int64(n), _p(lnw), C.c_int64(n),
                                C.c_double(ess_frac), C.byref(tr))
    return tr


def mdn_outputs(params, tr, x):
    """(z~ [n][7], network outputs [n][336]) of samples x[7][n]."""
    P = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[1]
    z = np.zeros((n, 7))
    o = np.zeros((n, 336))
    lib().orc_mdn_outputs(_p(P), C.byref(tr), _p(x), C.c_int64(n), C.c_int64(n), _p(z), _p(o))
    return z, o
