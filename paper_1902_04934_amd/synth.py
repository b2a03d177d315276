"""Seeded synthetic inputs for the ILE hot path.

This module is the one source of inputs shared by the HIP path and the CPU
oracle.  It holds none of the method's arithmetic (no antenna patterns, no
harmonics, no delays, no likelihood): only stand-in series for Q_k,lm, Gram
matrices for U_k and V_k, and extrinsic samples drawn from the prior.  It
imports nothing from the rest of the package.

The paper measures on zero-noise injections made with waveform models that
are not available here (Sec. III.A); the stand-ins keep the shapes of its
workloads: 2-3 L-shaped detectors, 4096 or 16384 Hz series, l=2..4 modes,
p(D) ~ D^2 up to 1 Gpc, blocks of extrinsic samples.

Q stand-in (one per detector k and mode a):
    Q[i] = A_a exp(-u^2 / 2 sigma_t^2) exp(i (phi_ka + 2 pi (f0 u + fdot u^2/2)))
           + n_i,   u = (i - i_k) dt,  n_i ~ CN(0, 1)
with sigma_t = 4 ms, f0 = 60 Hz, fdot = 4000 Hz/s, A_a = 20 * 0.3**a (a = the
position of the mode in MODE_ORDER), i_k = n_q/2 + delta_k where delta_k is a
seeded integer offset within +-8 ms (a stand-in for unequal arrival times).
U_k = A^H A / n_v, V_k = A^T A / n_v from one seeded complex Gaussian
matrix A (n_v = 64 rows), scaled so trace(U_k)/n_lm = mean_a A_a^2; using the
same A makes V complex-symmetric and the quadratic form non-negative.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0
EARTH_RADIUS_M = 6378.0e3

# (lat deg, lon deg, x-arm azimuth deg counter-clockwise from local East)
DETECTORS = {
    "D1": (46.455, -119.408, 126.0),
    "D2": (30.563, -90.774, 198.0),
    "D3": (43.631, 10.504, 71.0),
}

# Canonical mode order; configurations take prefixes of it (5, 9, 13, 21).
MODE_ORDER = [
    (2, 2), (2, -2), (2, 1), (2, -1), (2, 0),
    (3, 3), (3, -3), (3, 2), (3, -2),
    (4, 4), (4, -4), (4, 3), (4, -3),
    (3, 1), (3, -1), (3, 0), (4, 2), (4, -2), (4, 1), (4, -1), (4, 0),
]

D_REF_MPC = 100.0
D_MIN_MPC = 10.0
D_MAX_MPC = 1000.0
T_REF_MAX_S = 0.010


@dataclass
class Instance:
    """One intrinsic point: Q, U, V and the static configuration."""
    dets: list            # [(lat, lon, az)]
    modes: list           # [(l, m)]
    srate_hz: float
    n_t: int
    Q: np.ndarray         # complex128 [n_det][n_lm][n_q]
    U: np.ndarray         # complex128 [n_det][n_lm][n_lm]
    V: np.ndarray         # complex128 [n_det][n_lm][n_lm]
    d_ref_mpc: float = D_REF_MPC
    gmst_rad: float = 0.0
    earth_radius_m: float = EARTH_RADIUS_M
    t_ref_max_s: float = T_REF_MAX_S
    meta: dict = field(default_factory=dict)

    @property
    def n_det(self):
        return len(self.dets)

    @property
    def n_lm(self):
        return len(self.modes)

    @property
    def n_q(self):
        return self.Q.shape[-1]

    @property
    def t0_s(self):
        """Time of Q[0] relative to the geocentre event time."""
        return -(self.n_q // 2) / self.srate_hz


def make_instance(det_names, n_lm, n_q, srate_hz, n_t, seed, *,
                  noise=True, n_v=64):
    """Stand-in Q, U, V for one intrinsic point (recipe in the module doc)."""
    rng = np.random.default_rng(seed)
    dets = [DETECTORS[d] for d in det_names]
    modes = MODE_ORDER[:n_lm]
    n_det = len(dets)
    dt = 1.0 / srate_hz
    amp = 20.0 * 0.3 ** np.arange(n_lm)
    i = np.arange(n_q)
    Q = np.empty((n_det, n_lm, n_q), np.complex128)
    max_off = int(0.008 / dt)
    for k in range(n_det):
        ik = n_q // 2 + int(rng.integers(-max_off, max_off + 1))
        u = (i - ik) * dt
        env = np.exp(-u * u / (2 * 0.004 ** 2))
        chirp = 2 * np.pi * (60.0 * u + 0.5 * 4000.0 * u * u)
        for a in range(n_lm):
            ph = rng.uniform(0, 2 * np.pi)
            Q[k, a] = amp[a] * env * np.exp(1j * (ph + chirp))
            if noise:
                Q[k, a] += (rng.standard_normal(n_q) +
                            1j * rng.standard_normal(n_q)) / math.sqrt(2.0)
    U = np.empty((n_det, n_lm, n_lm), np.complex128)
    V = np.empty((n_det, n_lm, n_lm), np.complex128)
    target = float(np.mean(amp ** 2))
    for k in range(n_det):
        A = (rng.standard_normal((n_v, n_lm)) +
             1j * rng.standard_normal((n_v, n_lm))) / math.sqrt(2.0)
        Uk = A.conj().T @ A / n_v
        Vk = A.T @ A / n_v
        s = target / (np.trace(Uk).real / n_lm)
        U[k] = 0.5 * (Uk + Uk.conj().T) * s      # exactly Hermitian
        V[k] = 0.5 * (Vk + Vk.T) * s             # exactly symmetric
    return Instance(dets=dets, modes=modes, srate_hz=float(srate_hz),
                    n_t=int(n_t), Q=Q, U=U, V=V,
                    meta=dict(seed=seed, det_names=list(det_names)))


def prior_samples(n, seed, *, d_min=D_MIN_MPC, d_max=D_MAX_MPC,
                  t_ref_max=T_REF_MAX_S):
    """Extrinsic samples from the prior, SoA [7][n], and their log density.

    Prior: ra ~ U[0, 2pi); sin(dec) ~ U[-1, 1]; psi ~ U[0, pi);
    phi ~ U[0, 2pi); cos(iota) ~ U[-1, 1]; p(D) ~ D^2 on [d_min, d_max];
    t_ref ~ U[-t_ref_max, t_ref_max].  ln p is the density in the
    coordinates (ra, dec, psi, phi, cos iota, D, t_ref).
    """
    rng = np.random.default_rng(seed)
    s = np.empty((7, n), np.float64)
    s[0] = rng.uniform(0, 2 * np.pi, n)
    s[1] = np.arcsin(rng.uniform(-1, 1, n))
    s[2] = rng.uniform(0, np.pi, n)
    s[3] = rng.uniform(0, 2 * np.pi, n)
    s[4] = rng.uniform(-1, 1, n)
    v3 = d_max ** 3 - d_min ** 3
    s[5] = np.cbrt(d_min ** 3 + rng.uniform(0, 1, n) * v3)
    s[6] = rng.uniform(-t_ref_max, t_ref_max, n)
    ln_p = (-np.log(2 * np.pi) + np.log(np.cos(s[1]) / 2) - np.log(np.pi)
            - np.log(2 * np.pi) - np.log(2.0) + np.log(3 * s[5] ** 2 / v3)
            - np.log(2 * t_ref_max))
    return s, ln_p


# ------------------------------------------------------------- workloads
def config1(seed=None):
    """Plain ILE, one point: D1+D2, l=2 (5 modes), 4096 points at 4096 Hz,
    201 bins, 1e4 prior samples."""
    seed = 1001 if seed is None else seed
    return make_instance(["D1", "D2"], 5, 4096, 4096.0, 201, seed)


def config2(seed=None):
    """Plain ILE at scale: D1+D2+D3, l=2..4 (21 modes), 16384 points at
    16384 Hz, 1601 bins, 1e6 prior samples."""
    seed = 2001 if seed is None else seed
    return make_instance(["D1", "D2", "D3"], 21, 16384, 16384.0, 1601, seed)


CONFIG_SAMPLES = {1: (10_000, 1002), 2: (1_000_000, 2002)}


def batched_point(p, *, n_q=16384, srate_hz=16384.0):
    """Point p of the batched workload: 3 detectors, n_lm in {5, 9, 13, 21}
    and n_t = 2h+1 with h ~ U{100..800}, both chosen by the point's seed."""
    seed = 100_000 + p
    rng = np.random.default_rng(seed)
    n_lm = int(rng.choice([5, 9, 13, 21]))
    n_t = 2 * int(rng.integers(100, 801)) + 1
    return make_instance(["D1", "D2", "D3"], n_lm, n_q, srate_hz, n_t,
                         seed + 7_000_000)


# ------------------------------------------------- learned-proposal inputs
MDN_BLOCKS = [  # (name, size, fan_in, fan_out) of the flat parameter vector
    ("W1", 128 * 7, 7, 128), ("b1", 128, 0, 0),
    ("W2", 128 * 128, 128, 128), ("b2", 128, 0, 0),
    ("W3", 336 * 128, 128, 336), ("b3", 336, 0, 0),
]


def mdn_params(seed, *, gain=1.0, bias=0.3):
    """A seeded parameter vector for the mixture-density proposal (float32,
    60880 values in the block order of MDN_BLOCKS): Glorot-uniform weights
    times gain, uniform biases in [-bias, bias].  Plain random numbers; the
    masks are applied by whoever evaluates the network."""
    rng = np.random.default_rng(seed)
    out = []
    for _, size, fi, fo in MDN_BLOCKS:
        if fi:
            a = gain * math.sqrt(6.0 / (fi + fo))
            out.append(rng.uniform(-a, a, size))
        else:
            out.append(rng.uniform(-bias, bias, size))
    return np.concatenate(out).astype(np.float32)


# ------------------------------------------------ injection inputs
def mode_waveforms(modes, n_q, srate_hz, seed, *, sigma_t=0.03, f0=40.0, fdot=1500.0,
                   amp=1.0):
    """Stand-in mode series h_lm[i] (complex [n_lm][n_q]) for a zero-noise
    injection, in place of the paper's waveform models (Sec. III.A): a
    Gaussian-enveloped chirp centred on sample 0 (circular time u = i dt,
    wrapped to [-n_q/2, n_q/2) dt) whose phase advances m/2 times a common
    chirp phase (the m-dependence of the modes), with mode amplitudes
    amp * 0.3**rank and a seeded phase offset per mode.  Data only."""
    rng = np.random.default_rng(seed)
    dt = 1.0 / srate_hz
    i = np.arange(n_q)
    u = np.where(i < n_q // 2, i, i - n_q) * dt
    env = np.exp(-u * u / (2 * sigma_t ** 2))
    chirp = 2 * np.pi * (f0 * u + 0.5 * fdot * u * u)
    h = np.zeros((len(modes), n_q), np.complex128)
    for a, (l, m) in enumerate(modes):
        ph = rng.uniform(0, 2 * np.pi)
        h[a] = amp * 0.3 ** a * env * np.exp(1j * (ph + 0.5 * m * chirp))
    return h


def fd_inputs(det_names, n_lm, n_q, srate_hz, seed, *, f_knee=40.0):
    """Frequency-domain stand-ins for building Q, U, V: the stand-in mode
    series' transforms h_f [n_lm][n_q] (dt times the FFT; time origin at
    sample 0), per-detector data transforms d_f [n_det][n_q] (coloured
    Gaussian noise plus the first mode delayed by a seeded few ms and
    scaled), and a smooth coloured spectrum psd [n_det][n_q] at |f_i|
    (seismic wall below f_knee, flat bucket, shot-noise rise), each
    detector's scaled by a seeded factor.  Data only."""
    rng = np.random.default_rng(seed)
    modes = MODE_ORDER[:n_lm]
    dt = 1.0 / srate_hz
    h = mode_waveforms(modes, n_q, srate_hz, seed + 1, amp=20.0)
    h_f = dt * np.fft.fft(h, axis=1)
    df = srate_hz / n_q
    i = np.arange(n_q)
    f = np.abs(np.where(i < n_q // 2, i, i - n_q) * df)
    fs = np.maximum(f, df)
    shape = (f_knee / fs) ** 4 + 1.0 + (fs / (8 * f_knee)) ** 2
    n_det = len(det_names)
    psd = np.empty((n_det, n_q))
    d_f = np.empty((n_det, n_q), np.complex128)
    sf = np.where(i < n_q // 2, i, i - n_q) * df
    for k in range(n_det):
        psd[k] = 1e-3 * shape * rng.uniform(0.5, 2.0)
        noise = (rng.standard_normal(n_q) + 1j * rng.standard_normal(n_q)) \
            * np.sqrt(psd[k] / (4 * df))
        lag = rng.uniform(-0.01, 0.01)
        d_f[k] = noise + rng.uniform(0.5, 1.5) * h_f[0] * np.exp(-2j * np.pi * sf * lag)
    return dict(det_names=list(det_names), dets=[DETECTORS[d] for d in det_names],
                modes=modes, n_q=n_q, srate_hz=srate_hz, df=df, h_f=h_f, d_f=d_f, psd=psd)


CONFIG4_SEEDS = (4001, 4002)   # (data and injection, samples)


def combined_point(p):
    """Point p of the combined workload: the batched mix (3 detectors,
    n_lm in {5, 9, 13, 21}, n_t = 2h+1 with h ~ U{100..800}, 16384 points
    at 16384 Hz, all by the point's seed) with a zero-noise injection at
    network SNR 20 of the stand-in waveforms at seeded parameters, as for
    the learned-proposal workload.  Returns the pieces (see config4_parts)."""
    seed = 500_000 + p
    rng = np.random.default_rng(seed)
    n_lm = int(rng.choice([5, 9, 13, 21]))
    n_t = 2 * int(rng.integers(100, 801)) + 1
    names = ["D1", "D2", "D3"]
    modes = MODE_ORDER[:n_lm]
    n_q, srate = 16384, 16384.0
    theta = np.array([rng.uniform(0, 2 * np.pi), math.asin(rng.uniform(-1, 1)),
                      rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi),
                      rng.uniform(-1, 1), 400.0, rng.uniform(-0.5, 0.5) * T_REF_MAX_S])
    h = mode_waveforms(modes, n_q, srate, seed + 1, amp=20.0)
    return dict(det_names=names, dets=[DETECTORS[d] for d in names], modes=modes,
                n_q=n_q, srate_hz=srate, n_t=n_t, h_lm=h, theta_inj=theta, snr=20.0)


def lambda_sequence(n_points, seed=None, step=0.01):
    """A sequence of neighbouring intrinsic points for proposal reuse: the
    learned-proposal workload's detectors, modes, grid and injected extrinsic
    parameters, with the stand-in chirp's f0 and fdot (its intrinsic
    parameters) raised by step * p at point p.  Each point is its own
    zero-noise injection at network SNR 20, so neighbouring points share the
    extrinsic posterior's location.  Returns a list of parts."""
    base = config4_parts(seed)
    seed = CONFIG4_SEEDS[0] if seed is None else seed
    out = []
    for p in range(n_points):
        s = 1.0 + step * p
        h = mode_waveforms(base["modes"], base["n_q"], base["srate_hz"], seed + 1, amp=20.0,
                           f0=40.0 * s, fdot=1500.0 * s)
        out.append(dict(base, h_lm=h))
    return out


def config4_parts(seed=None):
    """Learned-proposal workload: 3 detectors, 9 modes (l = 2, 3), 16384
    points at 16384 Hz, 1601 bins; a zero-noise injection at network SNR 20
    of the stand-in waveforms at seeded parameters (distance set by the SNR).
    Returns the pieces; the injection itself (responses, Q, U, V) is built by
    whoever evaluates it."""
    seed = CONFIG4_SEEDS[0] if seed is None else seed
    rng = np.random.default_rng(seed)
    names = ["D1", "D2", "D3"]
    modes = MODE_ORDER[:9]
    n_q, srate, n_t = 16384, 16384.0, 1601
    theta = np.array([rng.uniform(0, 2 * np.pi), math.asin(rng.uniform(-1, 1)),
                      rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi),
                      rng.uniform(-1, 1), 400.0, rng.uniform(-0.5, 0.5) * T_REF_MAX_S])
    h = mode_waveforms(modes, n_q, srate, seed + 1, amp=20.0)
    return dict(det_names=names, dets=[DETECTORS[d] for d in names], modes=modes,
                n_q=n_q, srate_hz=srate, n_t=n_t, h_lm=h, theta_inj=theta, snr=20.0)
