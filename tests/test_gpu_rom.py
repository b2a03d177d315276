"""GPU parity of the surrogate (linear-basis) form (Sec. V: one Monte Carlo
over intrinsic and extrinsic parameters at once) against the oracle's
definition, through the C ABI (ile_rom_set, ile_rom_eval_dev,
ile_rom_integrate_dev).

The oracle rebuilds Q, U, V at each sample's lambda and evaluates Eq. (7)
and Eq. (9); the device forms z = C(lambda) Y per sample and runs the
contraction over the basis.  Same tolerances as the plain path: 1e-9 absolute
per sample in FP64 (the two sum the basis in different orders), 1e-4 relative
in FP32; ln L_marg within 1e-9 in FP64.
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


@pytest.fixture(scope="module")
def case(orc):
    from test_rom_pins import _case, _samples
    base, modes, A, E, data, basis, th, rng = _case(orc, seed=81)
    n = 700
    lams = rng.uniform(-1, 1, n)
    s8 = _samples(th, lams, rng, n)
    s8[:, ::7] = np.vstack([synth.prior_samples(100, 82)[0], rng.uniform(-1, 1, (1, 100))])
    want = orc.rom_eval(basis, modes, A, s8)
    return basis, modes, A, s8, want


def _run(torch, ctx, s8, ln_p=None, ln_q=None, integrate=False):
    S = torch.tensor(np.ascontiguousarray(s8), device="cuda")
    n = s8.shape[1]
    torch.cuda.synchronize()
    if integrate:
        P = torch.tensor(ln_p, device="cuda")
        Qd = torch.tensor(ln_q, device="cuda")
        r = torch.zeros(6, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ile.ile_rom_integrate_dev(ctx.h, S, P, Qd, n, r)
        ctx.sync()
        return r.cpu().numpy()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ile.ile_rom_eval_dev(ctx.h, S, n, out)
    ctx.sync()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_rom_eval_matches_oracle(torch, orc, case, precision, tol):
    basis, modes, A, s8, want = case
    with ile.Context(basis, precision=precision) as ctx:
        ile.ile_rom_set(ctx.h, modes, A)
        got = _run(torch, ctx, s8)
        # the plain path on the same context is unaffected
        plain = ctx.eval(s8[:7, :50])
    err = np.abs(got - want) / (np.maximum(1.0, np.abs(want)) if precision != "fp64" else 1.0)
    print(f"rom {precision}: max err {err.max():.3e} over {s8.shape[1]} samples")
    assert err.max() <= tol
    ref = orc.Ctx(basis).eval(s8[:7, :50])
    assert np.abs(plain - ref).max() <= (1e-9 if precision == "fp64" else 1e-3 * np.abs(ref).max())


def test_rom_integrate_matches_oracle(torch, orc, case):
    basis, modes, A, s8, want = case
    rng = np.random.default_rng(83)
    n = s8.shape[1]
    lp = rng.normal(0, 1, n)
    lq = rng.normal(0, 1, n)
    ref = orc.integrate(want, lp, lq)
    with ile.Context(basis) as ctx:
        ile.ile_rom_set(ctx.h, modes, A)
        r = _run(torch, ctx, s8, lp, lq, integrate=True)
    assert abs(r[0] - ref["ln_L_marg"]) <= 1e-9
    assert abs(r[1] - ref["n_eff"]) <= 1e-9 * ref["n_eff"]
    assert r[5] == n


def test_rom_full_size_sampled(torch, orc):
    """The benchmark point's shape as a surrogate: 21 basis functions, 3
    detectors, Q 16384 points, 1601 bins, 21 physical modes, 4 powers of
    lambda, 10^6 joint samples; 40 sampled outputs against the oracle."""
    basis = synth.config2()
    modes = synth.MODE_ORDER[:21]
    rng = np.random.default_rng(84)
    A = (rng.normal(size=(21, 21, 4)) + 1j * rng.normal(size=(21, 21, 4))) / 21
    n = 1_000_000
    s, _ = synth.prior_samples(n, 85)
    s8 = np.vstack([s, rng.uniform(-1, 1, (1, n))])
    with ile.Context(basis) as ctx:
        ile.ile_rom_set(ctx.h, modes, A)
        got = _run(torch, ctx, s8)
        ms = ctx.last_kernel_ms()
    idx = rng.choice(n, 40, replace=False)
    want = orc.rom_eval(basis, modes, A, s8[:, idx])
    err = np.abs(got[idx] - want).max()
    print(f"rom full size: contraction {ms:.2f} ms, sampled max err {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= 1e-9


def test_rom_errors(torch, case):
    basis, modes, A, s8, _ = case
    with ile.Context(basis) as ctx:
        S = torch.tensor(np.ascontiguousarray(s8[:, :10]), device="cuda")
        out = torch.zeros(10, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(ile.IleError) as e:
            ile.ile_rom_eval_dev(ctx.h, S, 10, out)
        assert e.value.status == ile.ILE_E_STATE
        with pytest.raises(ile.IleError) as e:
            ile.ile_rom_set(ctx.h, [(1, 0)] + list(modes[1:]), A)
        assert e.value.status == ile.ILE_E_ARG
        ile.ile_rom_set(ctx.h, modes, A)
        bad = s8[:, :10].copy()
        bad[7, 3] = 1.5
        with pytest.raises(ile.IleError) as e:
            _run(torch, ctx, bad)
        assert e.value.status == ile.ILE_E_RANGE
        # the context recovers
        got = _run(torch, ctx, s8[:, :10])
        assert np.all(np.isfinite(got))


def test_rom_table_beyond_lds(torch, orc):
    """32 physical modes (l = 2..5), 21 basis functions and 8 powers of
    lambda: the coefficient table (86 KB) does not fit the 64 KB staging
    limit, so k_rom_z reads it from global memory."""
    basis = synth.make_instance(["D1", "D2", "D3"], 21, 4096, 4096.0, 201, 86)
    modes = [(l, m) for l in range(2, 6) for m in range(-l, l + 1)]
    assert len(modes) == 32
    rng = np.random.default_rng(87)
    A = (rng.normal(size=(32, 21, 8)) + 1j * rng.normal(size=(32, 21, 8))) / 32
    s, _ = synth.prior_samples(300, 88)
    s8 = np.vstack([s, rng.uniform(-1, 1, (1, 300))])
    with ile.Context(basis) as ctx:
        ile.ile_rom_set(ctx.h, modes, A)
        got = _run(torch, ctx, s8)
    want = orc.rom_eval(basis, modes, A, s8)
    err = np.abs(got - want).max()
    print(f"rom, table in global memory: max err {err:.3e}")
    assert err <= 1e-9
