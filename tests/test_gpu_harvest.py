"""GPU parity of the extrinsic harvest (Sec. V; Eq. (3) at fixed intrinsic
parameters) against the oracle's two-stage inverse-CDF draw, through the C
ABI (ile_harvest_dev).

The sample index and the bin are integers and must equal the oracle's.  Two
results are both correct only where the target (uniform times total) falls
within rounding of a boundary of the cumulative weights: the FP64 per-sample
values differ from the oracle's by at most 1e-9 and the per-bin ones by about
1e-13 relative, and the two sides sum in different orders.  A pick that
differs from the oracle's must therefore be valid on the oracle's cumulative
weights to within 1e-8 of the total (sample) or 1e-10 (bin), and be a
positive weight.  The harvested parameters equal the chosen sample's, with
row 6 the bin time t_ref + (j - (n_t-1)/2)/srate, bit for bit.
"""
import numpy as np
import pytest

from paper_1902_04934_amd import ile, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


def _dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def run_harvest(torch, ctx, s, lp, lq, u, with_theta=True):
    n, n_out = s.shape[1], u.shape[1]
    S, P, Q, U = (_dev(torch, x) for x in (s, lp, lq, u))
    idx = torch.full((max(n_out, 1),), -7, dtype=torch.int64, device="cuda")
    bins = torch.full((max(n_out, 1),), -7, dtype=torch.int32, device="cuda")
    th = torch.full((7, max(n_out, 1)), np.nan, dtype=torch.float64, device="cuda") \
        if with_theta else None
    torch.cuda.synchronize()   # the fills above run on torch's stream, not the context's
    ctx.harvest_dev(S, P, Q, n, U, n_out, idx, bins, th)
    torch.cuda.synchronize()
    return (idx.cpu().numpy()[:n_out], bins.cpu().numpy()[:n_out],
            th.cpu().numpy()[:, :n_out] if with_theta else None)


def _valid(c, target, i, tol):
    lo = c[i - 1] if i > 0 else 0.0
    return c[i] > lo and lo - tol * c[-1] <= target <= c[i] + tol * c[-1]


def check_samples(orc, s, lp, lq, lnL_or, u0, idx, tol=1e-8):
    """Sample picks against the oracle's cumulative weights; returns the
    number of picks that differ (each checked valid)."""
    lw = lnL_or + lp - lq
    lw = np.where(np.isfinite(lw), lw, -np.inf)
    c = np.cumsum(np.exp(lw - lw.max()))
    diff = 0
    for k in range(idx.size):
        t = u0[k] * c[-1]
        want = orc.inverse_cdf(c, t)
        if idx[k] != want:
            diff += 1
            assert _valid(c, t, int(idx[k]), tol), (k, int(idx[k]), want)
    return diff


def check_bins(orc, octx, inst, s, idx, bins, theta, u1, ks, tol=1e-10):
    h = (inst.n_t - 1) // 2
    diff = 0
    for k in ks:
        a = int(idx[k])
        L = octx.lnL_series(s[:, a])
        c = np.cumsum(np.exp(L - L.max()))
        t = u1[k] * c[-1]
        want = orc.inverse_cdf(c, t)
        if bins[k] != want:
            diff += 1
            assert _valid(c, t, int(bins[k]), tol), (k, int(bins[k]), want)
    if theta is not None:
        assert np.array_equal(theta[:6], s[:6, idx])
        assert np.array_equal(theta[6], s[6, idx] + (bins.astype(np.int64) - h) / inst.srate_hz)
    return diff


def _inputs(n, seed, n_out, q_spread=0.5):
    s, lp = synth.prior_samples(n, seed)
    rng = np.random.default_rng(seed + 1)
    lq = lp + rng.normal(0.0, q_spread, n)
    u = rng.uniform(size=(2, n_out))
    return s, lp, lq, u


@pytest.mark.parametrize("n,n_out", [(3001, 3000), (257, 64), (1, 5)])
def test_harvest_parity_fp64(torch, orc, n, n_out):
    inst = synth.make_instance(["D1", "D2", "D3"], 9, 4096, 4096.0, 201, 501)
    s, lp, lq, u = _inputs(n, 502, n_out)
    octx = orc.Ctx(inst)
    lnL = octx.eval(s)
    with ile.Context(inst) as ctx:
        idx, bins, theta = run_harvest(torch, ctx, s, lp, lq, u)
    assert idx.min() >= 0 and idx.max() < n and bins.min() >= 0 and bins.max() < inst.n_t
    d1 = check_samples(orc, s, lp, lq, lnL, u[0], idx)
    d2 = check_bins(orc, octx, inst, s, idx, bins, theta, u[1], range(n_out))
    print(f"harvest fp64 N={n} n_out={n_out}: {d1} sample and {d2} bin picks differ (valid)")
    assert d1 + d2 <= max(1, n_out // 1000)


def test_harvest_matches_oracle_harvest(torch, orc):
    """Same inputs through the oracle's own harvest: identical picks."""
    inst = synth.make_instance(["D1", "D2", "D3"], 5, 2048, 2048.0, 101, 511)
    s, lp, lq, u = _inputs(700, 512, 500)
    i_or, b_or, th_or = orc.harvest(orc.Ctx(inst), s, lp, lq, u)
    with ile.Context(inst) as ctx:
        idx, bins, theta = run_harvest(torch, ctx, s, lp, lq, u)
    same = (idx == i_or) & (bins == b_or)
    assert same.mean() > 0.99
    assert np.array_equal(theta[:, same], th_or[:, same])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_harvest_reduced_precision_valid(torch, orc, precision):
    """FP32/BF16 contraction: every pick is a valid draw of the oracle's
    weights perturbed by the reduced precision's own per-sample error.

    The context's per-sample ln L_margT differs from the FP64 oracle's by
    delta_i, |delta_i| <= 1e-4 max(1, |ln L|) (the precision forms' bound,
    asserted here).  Weights exp(ln w + delta) move every cumulative sum and
    the target by a factor within exp(+-max|delta|), so a pick that differs
    from the oracle's must be valid on the oracle's cumulative weights within
    expm1(2 max|delta|) of the total.  The bins get the same check with the
    bound itself in place of a measured delta (1e-4 of the row's largest
    |L|)."""
    inst = synth.make_instance(["D1", "D2", "D3"], 9, 4096, 4096.0, 201, 521)
    s, lp, lq, u = _inputs(2000, 522, 2000)
    octx = orc.Ctx(inst)
    lnL = octx.eval(s)
    lw = lnL + lp - lq
    c = np.cumsum(np.exp(lw - lw.max()))
    with ile.Context(inst, precision=precision) as ctx:
        got = ctx.eval(s)
        idx, bins, theta = run_harvest(torch, ctx, s, lp, lq, u)
    delta = np.abs(got - lnL)
    assert np.all(delta <= 1e-4 * np.maximum(1.0, np.abs(lnL)))
    tol = np.expm1(2.0 * 1.5 * delta.max()) + 1e-12
    w = np.diff(np.concatenate([[0.0], c]))
    assert np.all(w[idx] > 0)
    d1 = check_samples(orc, s, lp, lq, lnL, u[0], idx, tol=tol)
    h = (inst.n_t - 1) // 2
    d2 = 0
    for k in range(0, 2000, 10):
        a = int(idx[k])
        L = octx.lnL_series(s[:, a])
        cj = np.cumsum(np.exp(L - L.max()))
        t = u[1, k] * cj[-1]
        if bins[k] != orc.inverse_cdf(cj, t):
            d2 += 1
            tb = np.expm1(2.0 * 1e-4 * max(1.0, np.abs(L).max()))
            assert _valid(cj, t, int(bins[k]), tb), (k, int(bins[k]))
    print(f"harvest {precision}: max |d lnL| {delta.max():.2e}, {d1} of 2000 sample picks and "
          f"{d2} of 200 bin picks differ (all valid)")
    assert np.array_equal(theta[:6], s[:6, idx])
    assert np.array_equal(theta[6], s[6, idx] + (bins.astype(np.int64) - h) / inst.srate_hz)


def test_harvest_chunks_and_full_size(torch, orc):
    """1601 bins, 21 modes, 3 detectors, 10^6 prior samples, 10^5 draws
    in one series chunk: every sample pick against
    the oracle's cumulative weights over all 10^6 samples, bins sampled
    (300 random draws)."""
    inst = synth.config2()
    n, seed = synth.CONFIG_SAMPLES[2]
    n_out = 100_000
    s, lp = synth.prior_samples(n, seed)
    rng = np.random.default_rng(seed + 5)
    lq = lp.copy()
    u = rng.uniform(size=(2, n_out))
    print("harvest full size: oracle eval of 1e6 samples", flush=True)
    octx = orc.Ctx(inst)
    lnL = octx.eval(s)
    with ile.Context(inst) as ctx:
        idx, bins, theta = run_harvest(torch, ctx, s, lp, lq, u)
    d1 = check_samples(orc, s, lp, lq, lnL, u[0], idx)
    m_max = (1 << 31) // (inst.n_t * 8)
    ks = set(rng.choice(n_out, 300, replace=False).tolist())
    for b in range(m_max, n_out, m_max):
        ks |= {b - 1, b}
    ks = sorted(ks)
    d2 = check_bins(orc, octx, inst, s, idx, bins, None, u[1], ks)
    h = (inst.n_t - 1) // 2
    assert np.array_equal(theta[:6], s[:6, idx])
    assert np.array_equal(theta[6], s[6, idx] + (bins.astype(np.int64) - h) / inst.srate_hz)
    print(f"harvest full: {len(np.unique(idx))} distinct samples drawn; "
          f"{d1} sample and {d2} bin picks differ (valid)")
    assert d1 <= n_out // 1000 and d2 <= 2


def test_harvest_result_is_the_integral(torch, orc):
    """The optional Eq. (4) result of the harvest's own evaluation equals
    ile_integrate_dev's on the same samples (same kernels: bit for bit) and
    the oracle's reduction to 1e-9."""
    inst = synth.make_instance(["D1", "D2", "D3"], 9, 4096, 4096.0, 201, 551)
    s, lp, lq, u = _inputs(2500, 552, 300)
    want = orc.integrate(orc.Ctx(inst).eval(s), lp, lq)
    with ile.Context(inst) as ctx:
        S, P, Q, U = (_dev(torch, x) for x in (s, lp, lq, u))
        idx = torch.empty(300, dtype=torch.int64, device="cuda")
        bins = torch.empty(300, dtype=torch.int32, device="cuda")
        r1 = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
        r2 = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ctx.harvest_dev(S, P, Q, s.shape[1], U, 300, idx, bins, None, r1)
        ctx.integrate_dev(S, P, Q, s.shape[1], r2)
        ctx.sync()
        a, b = r1.cpu().numpy(), r2.cpu().numpy()
    assert np.array_equal(a, b)
    assert abs(a[0] - want["ln_L_marg"]) <= 1e-9
    assert abs(a[1] - want["n_eff"]) <= 1e-9 * want["n_eff"]
    assert a[5] == s.shape[1]


def test_harvest_chunked_series(torch, orc):
    """Series held for at most 777 draws at a time (ILE_OPT_HARVEST_ROWS):
    the same picks as one chunk, and both sides of every chunk boundary
    against the oracle."""
    inst = synth.make_instance(["D1", "D2", "D3"], 9, 4096, 4096.0, 2401, 541)
    s, lp, lq, u = _inputs(1500, 542, 5000)
    octx = orc.Ctx(inst)
    with ile.Context(inst) as ctx:
        one = run_harvest(torch, ctx, s, lp, lq, u)
        ile.ile_set_option(ctx.h, ile.ILE_OPT_HARVEST_ROWS, 777)
        many = run_harvest(torch, ctx, s, lp, lq, u)
    for x, y in zip(one, many):
        assert np.array_equal(x, y)
    ks = sorted({k for b in range(777, 5000, 777) for k in (b - 1, b)} | {0, 4999})
    check_bins(orc, octx, inst, s, many[0], many[1], many[2], u[1], ks)


def test_harvest_edge_cases(torch, orc):
    inst = synth.make_instance(["D1", "D2"], 5, 2048, 2048.0, 51, 531)
    s, lp, lq, u = _inputs(40, 532, 30)
    with ile.Context(inst) as ctx:
        # n_out = 0 is a no-op
        idx, bins, _ = run_harvest(torch, ctx, s, lp, lq, u[:, :0])
        assert idx.size == 0
        # only one positive weight: always that sample; theta may be NULL
        lp1 = np.full(40, -np.inf)
        lp1[17] = 0.0
        idx, bins, th = run_harvest(torch, ctx, s, lp1, lq, u, with_theta=False)
        assert np.all(idx == 17) and th is None
        # u = 0 takes the first positive weight
        idx, _, _ = run_harvest(torch, ctx, s, lp1, lq, np.zeros((2, 3)))
        assert np.all(idx == 17)
        for bad_u in (1.0, -0.25, np.nan):
            ub = u.copy()
            ub[1, 4] = bad_u
            with pytest.raises(ile.IleError) as e:
                run_harvest(torch, ctx, s, lp, lq, ub)
            assert e.value.status == ile.ILE_E_RANGE
        lqb = lq.copy()
        lqb[3] = np.nan
        with pytest.raises(ile.IleError) as e:
            run_harvest(torch, ctx, s, lp, lqb, u)
        assert e.value.status == ile.ILE_E_RANGE
        with pytest.raises(ile.IleError) as e:
            run_harvest(torch, ctx, s, np.full(40, -np.inf), lq, u)
        assert e.value.status == ile.ILE_E_NUMERIC
        sb = s.copy()
        sb[6, 9] = 1.0   # t_ref far outside the window bound
        with pytest.raises(ile.IleError) as e:
            run_harvest(torch, ctx, sb, lp, lq, u)
        assert e.value.status == ile.ILE_E_RANGE
        # the context still works after errors, and repeats are identical
        a = run_harvest(torch, ctx, s, lp, lq, u)
        b = run_harvest(torch, ctx, s, lp, lq, u)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        lnL = orc.Ctx(inst).eval(s)
        check_samples(orc, s, lp, lq, lnL, u[0], a[0])


def test_harvest_single_bin(torch, orc):
    """n_t = 1: every draw takes bin 0 and keeps its sample's t_ref; the
    sample picks still follow the oracle."""
    inst = synth.make_instance(["D1", "D2"], 3, 1024, 1024.0, 1, 541)
    s, lp, lq, u = _inputs(90, 542, 40)
    with ile.Context(inst) as ctx:
        idx, bins, theta = run_harvest(torch, ctx, s, lp, lq, u)
    assert np.all(bins == 0)
    assert np.array_equal(theta, s[:, idx])
    check_samples(orc, s, lp, lq, orc.Ctx(inst).eval(s), u[0], idx)
