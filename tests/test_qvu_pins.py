"""Pins of the oracle's frequency-domain Q, U, V (Eq. (2) and Eq. (8) as sums
over the FFT grid) against what the mathematics fixes:

* white noise, full band: Parseval and the correlation theorem make them
  equal to the time-domain construction of the injection instance (circular
  correlation in time, an independent route), for Q at every lag, U and V;
* a single spectral line: closed forms, and zero outside the band;
* U is Hermitian and V complex-symmetric for any spectrum even in f.
"""
import numpy as np

from paper_1902_04934_amd import synth


def _white_case(orc, n=256, seed=41):
    from test_oracle_pins import chirp_modes, random_theta
    rng = np.random.default_rng(seed)
    base = synth.make_instance(["D1", "D2", "D3"], 5, n, float(n), 11, seed)
    h = chirp_modes(base.n_lm, n, rng, base.srate_hz)
    inst, data, _ = orc.injection_instance(base, h, random_theta(rng), 0.3, rng)
    dt = 1.0 / base.srate_hz
    df = 1.0 / (n * dt)
    # the instance's Q[s] is the lag-s correlation and its t0 is -(n/2) dt:
    # the template's time origin sits n/2 samples into h
    h_f = dt * np.fft.fft(np.roll(h, -(n // 2), axis=1), axis=1)
    d_f = dt * np.fft.fft(data, axis=1)
    psd = np.full((base.n_det, n), 2.0 * dt)   # two-sided white: <a|b> = sum conj(a) b
    return inst, h_f, d_f, psd, df


def test_white_noise_equals_time_domain(orc):
    inst, h_f, d_f, psd, df = _white_case(orc)
    Q, U, V = orc.qvu_fd(h_f, d_f, psd, df, -1.0, np.inf, inst.t0_s)
    scale = np.abs(inst.Q).max()
    assert np.abs(Q - inst.Q).max() <= 1e-11 * scale
    assert np.abs(U - inst.U).max() <= 1e-11 * np.abs(inst.U).max()
    assert np.abs(V - inst.V).max() <= 1e-11 * np.abs(inst.V).max()


def test_sampled_lags_match_full(orc):
    inst, h_f, d_f, psd, df = _white_case(orc, n=128, seed=42)
    Q, _, _ = orc.qvu_fd(h_f, d_f, psd, df, -1.0, np.inf, inst.t0_s)
    s = np.array([0, 5, 63, 127])
    Qs, _, _ = orc.qvu_fd(h_f, d_f, psd, df, -1.0, np.inf, inst.t0_s, s_idx=s)
    assert np.array_equal(Qs, Q[:, :, s])


def test_single_line_closed_form_and_band(orc):
    n, df, t0 = 64, 0.5, -3.1
    f = orc.fft_freqs(n, df)
    rng = np.random.default_rng(7)
    for j in (3, 40, 0, 32):
        h_f = np.zeros((2, n), complex)
        h_f[:, j] = [1.5 - 0.5j, 0.2 + 2j]
        d_f = (rng.normal(size=(1, n)) + 1j * rng.normal(size=(1, n)))
        psd = np.full((1, n), 0.7)
        # the band is open: a line exactly on either edge is outside it
        for f_min, f_max in ((-1.0, 1e9), (1.0, 10.0), (2.0, 40.0), (abs(f[j]), 1e9),
                             (-1.0, abs(f[j]))):
            Q, U, V = orc.qvu_fd(h_f, d_f, psd, df, f_min, f_max, t0)
            inside = f_min < abs(f[j]) < f_max
            t = t0 + np.arange(n) / (n * df)
            want = (2 * df / 0.7) * np.conj(h_f[:, j])[:, None] * d_f[0, j] \
                * np.exp(2j * np.pi * f[j] * t)[None, :]
            if inside:
                assert np.allclose(Q[0], want, rtol=1e-13, atol=1e-14)
                assert np.allclose(U[0], (2 * df / 0.7) * np.outer(np.conj(h_f[:, j]), h_f[:, j]),
                                   rtol=1e-14, atol=0)
            else:
                assert np.all(Q == 0) and np.all(U == 0)
            # V pairs f with -f: a single line at f != 0 (or Nyquist) has none
            if j not in (0, n // 2) or not inside:
                assert np.all(V == 0)


def test_symmetries(orc):
    n, df = 96, 0.25
    rng = np.random.default_rng(9)
    h_f = rng.normal(size=(4, n)) + 1j * rng.normal(size=(4, n))
    d_f = rng.normal(size=(2, n)) + 1j * rng.normal(size=(2, n))
    f = orc.fft_freqs(n, df)
    psd = np.stack([1.0 + np.abs(f) ** 2, 0.5 + np.abs(f)])
    _, U, V = orc.qvu_fd(h_f, d_f, psd, df, 0.3, 9.0, 0.0)
    assert np.allclose(U, np.conj(np.transpose(U, (0, 2, 1))), rtol=1e-14, atol=1e-14)
    assert np.allclose(V, np.transpose(V, (0, 2, 1)), rtol=1e-14, atol=1e-14)
    assert np.all(np.diagonal(U, axis1=1, axis2=2).real > 0)
