"""GPU parity of Q, U, V built from frequency-domain series (Eq. (2) and
Eq. (8) on the FFT grid; ile_qvu_fd_dev, ile_set_data_fd) against the
oracle's direct sums, through the C ABI.

Tolerance: the inverse FFT sums n terms in log2(n) rounded passes, so Q is
compared to 1e-12 of the largest |Q| of its row set; U and V (plain sums in
a different order) to 1e-12 of their largest entry.  At 16384 lags the
oracle's direct sum is taken at 64 sampled lags.
"""
import numpy as np
import pytest

from paper_1902_04934_amd import ile, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def _blank(c, n_t):
    n_lm, nd = len(c["modes"]), len(c["dets"])
    return synth.Instance(dets=c["dets"], modes=c["modes"], srate_hz=c["srate_hz"], n_t=n_t,
                          Q=np.zeros((nd, n_lm, c["n_q"]), complex),
                          U=np.zeros((nd, n_lm, n_lm), complex),
                          V=np.zeros((nd, n_lm, n_lm), complex))


def _dev_build(torch, ctx, c, f_min, f_max, t0):
    nd, nl, n = len(c["dets"]), len(c["modes"]), c["n_q"]
    H = torch.tensor(np.ascontiguousarray(c["h_f"]).view(np.float64), device="cuda")
    D = torch.tensor(np.ascontiguousarray(c["d_f"]).view(np.float64), device="cuda")
    P = torch.tensor(np.ascontiguousarray(c["psd"]), device="cuda")
    Q = torch.empty((nd, nl, 2 * n), dtype=torch.float64, device="cuda")
    U = torch.empty((nd, nl, 2 * nl), dtype=torch.float64, device="cuda")
    V = torch.empty((nd, nl, 2 * nl), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ile.ile_qvu_fd_dev(ctx.h, H, D, P, n, c["df"], f_min, f_max, t0, Q, U, V)
    ms = ctx.last_kernel_ms()
    cv = lambda T: T.cpu().numpy().view(np.complex128)
    return cv(Q), cv(U), cv(V), ms


def _check(orc, c, Q, U, V, f_min, f_max, t0, s_idx=None):
    Qo, Uo, Vo = orc.qvu_fd(c["h_f"], c["d_f"], c["psd"], c["df"], f_min, f_max, t0, s_idx)
    Qg = Q if s_idx is None else Q[:, :, s_idx]
    eq = np.abs(Qg - Qo).max() / np.abs(Qo).max()
    eu = np.abs(U - Uo).max() / np.abs(Uo).max()
    ev = np.abs(V - Vo).max() / np.abs(Vo).max()
    assert eq <= 1e-12 and eu <= 1e-12 and ev <= 1e-12, (eq, eu, ev)
    return eq, eu, ev


class _Handle:
    """A bare context (no data installed): the device builder needs only the
    detector and mode counts."""

    def __init__(self, c):
        self.h = ile.ile_create(c["dets"], c["modes"], c["srate_hz"], 1)

    def last_kernel_ms(self):
        return ile.lib().ile_last_kernel_ms(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        ile.ile_destroy(self.h)


@pytest.mark.parametrize("n_q,f_min,f_max,t0", [(256, 3.0, 100.0, -0.125), (512, -1.0, 1e9, 0.0),
                                               (2, -1.0, 1e9, 0.3), (1024, 10.0, 200.0, -0.4)])
def test_fd_build_matches_oracle(torch, orc, n_q, f_min, f_max, t0):
    c = synth.fd_inputs(["D1", "D2", "D3"], 5, n_q, float(n_q), 601 + n_q)
    with _Handle(c) as ctx:
        Q, U, V, _ = _dev_build(torch, ctx, c, f_min, f_max, t0)
    print(n_q, _check(orc, c, Q, U, V, f_min, f_max, t0))


@pytest.mark.parametrize("n_q", [1024, 2048, 4096, 8192, 32768])
def test_fd_lds_and_four_step_sizes(torch, orc, n_q):
    """The single-workgroup transform at its largest size (1024) and the
    four-step form with square and oblong factorizations, 64 sampled lags."""
    c = synth.fd_inputs(["D1", "D2"], 3, n_q, float(n_q), 631 + n_q)
    with _Handle(c) as ctx:
        Q, U, V, _ = _dev_build(torch, ctx, c, 8.0, 0.4 * n_q, -0.3)
    s = np.random.default_rng(n_q).choice(n_q, 64, replace=False)
    print(n_q, _check(orc, c, Q, U, V, 8.0, 0.4 * n_q, -0.3, s))


def test_fd_full_size_sampled(torch, orc):
    """21 modes, 3 detectors, 16384 lags at 16384 Hz, band 20-4000 Hz."""
    c = synth.fd_inputs(["D1", "D2", "D3"], 21, 16384, 16384.0, 611)
    t0 = -0.5
    with _Handle(c) as ctx:
        Q, U, V, ms = _dev_build(torch, ctx, c, 20.0, 4000.0, t0)
    s = np.random.default_rng(3).choice(16384, 64, replace=False)
    errs = _check(orc, c, Q, U, V, 20.0, 4000.0, t0, s)
    print(f"full size: inverse FFT {ms:.3f} ms, rel errors {errs}")


def test_set_data_fd_white_noise_is_the_injection(torch, orc):
    """White noise, full band: the device construction installs the time-domain
    injection's Q, U, V (independent route), and the evaluation on it equals
    the oracle's on that instance."""
    from test_oracle_pins import chirp_modes, random_theta
    rng = np.random.default_rng(41)
    n = 1024
    base = synth.make_instance(["D1", "D2", "D3"], 5, n, float(n), 21, 41)
    h = chirp_modes(base.n_lm, n, rng, base.srate_hz)
    inst, data, _ = orc.injection_instance(base, h, random_theta(rng), 0.3, rng)
    dt = 1.0 / base.srate_hz
    h_f = dt * np.fft.fft(np.roll(h, -(n // 2), axis=1), axis=1)
    d_f = dt * np.fft.fft(data, axis=1)
    psd = np.full((3, n), 2.0 * dt)
    with ile.Context(_blank(dict(dets=base.dets, modes=base.modes, srate_hz=base.srate_hz,
                                 n_q=n), base.n_t)) as ctx:
        Q, U, V = ile.ile_set_data_fd(ctx.h, h_f, d_f, psd, 1.0 / (n * dt), -1.0, np.inf,
                                      inst.t0_s, base.dets, want_data=True)
        s, _ = synth.prior_samples(500, 42)
        got = ctx.eval(s)
    assert np.abs(Q - inst.Q).max() <= 1e-11 * np.abs(inst.Q).max()
    assert np.abs(U - inst.U).max() <= 1e-11 * np.abs(inst.U).max()
    assert np.abs(V - inst.V).max() <= 1e-11 * np.abs(inst.V).max()
    want = orc.Ctx(inst).eval(s)
    assert np.abs(got - want).max() <= 1e-8 * max(1.0, np.abs(want).max())


def test_fd_errors(torch):
    c = synth.fd_inputs(["D1", "D2"], 3, 256, 256.0, 621)
    with ile.Context(_blank(c, 1)) as ctx:
        args = (c["h_f"], c["d_f"], c["psd"], c["df"], 5.0, 60.0, -0.5, c["dets"])
        ile.ile_set_data_fd(ctx.h, *args)
        with pytest.raises(ile.IleError) as e:
            ile.ile_set_data_fd(ctx.h, c["h_f"], c["d_f"], c["psd"], c["df"], 60.0, 5.0, -0.5,
                                c["dets"])
        assert e.value.status == ile.ILE_E_ARG
        bad = c["psd"].copy()
        bad[1, 10] = 0.0            # 10 Hz: inside the band
        with pytest.raises(ile.IleError) as e:
            ile.ile_set_data_fd(ctx.h, c["h_f"], c["d_f"], bad, c["df"], 5.0, 60.0, -0.5,
                                c["dets"])
        assert e.value.status == ile.ILE_E_NUMERIC
        bad[1, 10] = 1.0
        bad[1, 100] = 0.0           # 100 Hz: outside it, never read as a weight
        ile.ile_set_data_fd(ctx.h, c["h_f"], c["d_f"], bad, c["df"], 5.0, 60.0, -0.5, c["dets"])
        c3 = synth.fd_inputs(["D1", "D2"], 3, 96, 96.0, 622)
        with pytest.raises(ile.IleError) as e:
            ile.ile_set_data_fd(ctx.h, c3["h_f"], c3["d_f"], c3["psd"], c3["df"], 5.0, 30.0,
                                0.0, c3["dets"])
        assert e.value.status == ile.ILE_E_UNSUPPORTED


def test_fd_largest_shapes(torch, orc):
    """Four detectors and 32 modes (the library's limits) on a 2048-point
    grid: every lag, U and V against the oracle."""
    n = 2048
    rng = np.random.default_rng(641)
    modes = [(l, m) for l in range(2, 6) for m in range(-l, l + 1)]
    dets = [synth.DETECTORS[d] for d in ("D1", "D2", "D3")] + [(36.4, 137.3, 15.0)]
    f = np.abs(np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)) * 1.0
    c = dict(dets=dets, modes=modes, srate_hz=float(n), n_q=n, df=1.0,
             h_f=(rng.normal(size=(32, n)) + 1j * rng.normal(size=(32, n))) / np.sqrt(1 + f / 50),
             d_f=rng.normal(size=(4, n)) + 1j * rng.normal(size=(4, n)),
             psd=np.stack([0.5 + 1e-4 * f ** 2 * (k + 1) for k in range(4)]))
    with _Handle(c) as ctx:
        Q, U, V, _ = _dev_build(torch, ctx, c, 10.0, 900.0, -0.25)
    print("4 x 32:", _check(orc, c, Q, U, V, 10.0, 900.0, -0.25))
