"""Pins of the oracle's surrogate (reduced-order) form: h_lm(lambda; t) =
sum_b c_lm,b(lambda) e_b(t) with polynomial coefficients (Sec. V), whose
Eq. (8) quantities follow from the basis overlaps by linearity:

* identity surrogate (one basis function per mode, c = 1): the plain
  likelihood of the basis instance, exactly;
* a physically consistent instance built the long way (templates h_lm(lambda)
  assembled in the time domain, Q, U, V correlated directly against data
  injected at another lambda) equals the surrogate composition, for every
  sample and lambda (pins the conjugate on c in Q and the orders in U, V);
* a surrogate with a conjugate or transpose misplaced fails that check.
"""
import numpy as np

from paper_1902_04934_amd import synth


def _corr(h, d):
    """Q[s] = sum_i conj(h[(i - s) mod n]) d[i] (circular, white noise)."""
    return np.fft.ifft(np.conj(np.fft.fft(h)) * np.fft.fft(d))


def _direct_instance(base, modes, h, data):
    n_det = len(base.dets)
    Q = np.stack([np.stack([_corr(h[a], data[k]) for a in range(h.shape[0])])
                  for k in range(n_det)])
    U = np.stack([np.conj(h) @ h.T for _ in range(n_det)])
    V = np.stack([h @ h.T for _ in range(n_det)])
    return synth.Instance(dets=base.dets, modes=list(modes), srate_hz=base.srate_hz,
                          n_t=base.n_t, Q=Q, U=U, V=V)


def _case(orc, seed=71, n=1024, n_b=6, n_lm=3, P=3):
    from test_oracle_pins import chirp_modes
    rng = np.random.default_rng(seed)
    base = synth.make_instance(["D1", "D2", "D3"], n_lm, n, float(n), 21, seed)
    E = chirp_modes(n_b, n, rng, base.srate_hz)                 # basis e_b(t)
    A = (rng.normal(size=(n_lm, n_b, P)) + 1j * rng.normal(size=(n_lm, n_b, P))) / n_b
    modes = synth.MODE_ORDER[:n_lm]
    th_inj = np.array([1.1, 0.3, 0.7, 2.0, 0.4, 150.0, 0.0031])
    h_true = orc.rom_coeffs(A, 0.3) @ E
    _, data, _ = orc.injection_instance(base, h_true, th_inj, 0.5, rng)
    basis = _direct_instance(base, synth.MODE_ORDER[:n_b], E, data)
    return base, modes, A, E, data, basis, th_inj, rng


def _samples(th, lam, rng, n):
    s = np.repeat(th[:, None], n, axis=1)
    s[:5] += rng.normal(0, 0.2, (5, n))
    s[4] = np.clip(s[4], -1, 1)
    s[6] += rng.uniform(-3e-3, 3e-3, n)
    return np.vstack([s, np.asarray(lam, float)[None, :]])


def test_identity_surrogate_is_plain(orc):
    inst = synth.make_instance(["D1", "D2"], 4, 512, 512.0, 11, 72)
    A = np.zeros((4, 4, 2), complex)
    A[:, :, 0] = np.eye(4)
    rng = np.random.default_rng(73)
    s, _ = synth.prior_samples(12, 74)
    s8 = np.vstack([s, rng.uniform(-1, 1, (1, 12))])
    got = orc.rom_eval(inst, inst.modes, A, s8)
    assert np.array_equal(got, orc.Ctx(inst).eval(s))


def test_surrogate_equals_direct_construction(orc):
    base, modes, A, E, data, basis, th, rng = _case(orc)
    lams = rng.uniform(-1, 1, 16)
    s8 = _samples(th, lams, rng, 16)
    got = orc.rom_eval(basis, modes, A, s8)
    for i, lam in enumerate(lams):
        h = orc.rom_coeffs(A, lam) @ E
        want = orc.Ctx(_direct_instance(base, modes, h, data)).eval(s8[:7, i:i + 1])[0]
        assert abs(got[i] - want) <= 1e-9 * max(1.0, abs(want)), (i, got[i], want)


def test_misplaced_conjugate_is_caught(orc):
    """The same check fails for a surrogate composed with conj(c) in U moved
    to the other side (U_k = C^H-like order swapped)."""
    base, modes, A, E, data, basis, th, rng = _case(orc, seed=75)
    lam = 0.6
    s8 = _samples(th, np.full(6, lam), rng, 6)
    inst = orc.rom_instance(basis, modes, A, lam)
    C = orc.rom_coeffs(A, lam)
    inst.U = np.stack([C @ basis.U[k] @ np.conj(C).T for k in range(basis.n_det)])
    bad = orc.Ctx(inst).eval(s8[:7])
    h = C @ E
    want = orc.Ctx(_direct_instance(base, modes, h, data)).eval(s8[:7])
    assert np.max(np.abs(bad - want)) > 1e-3
