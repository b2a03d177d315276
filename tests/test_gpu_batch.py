"""GPU parity of the batched form (many intrinsic points with uneven mode
counts and window lengths in one graph-captured run) against the oracle,
point by point, plus graph replay determinism and the autotuner."""
import os

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
def points():
    return [synth.batched_point(p, n_q=8192, srate_hz=8192.0) for p in range(10)]


def _check_batch(b, pts, seed, n, tol, rel):
    from oracle import oracle as O
    res = b.run(seed, n)
    lnl = b.lnL(n)
    for p, inst in enumerate(pts):
        s, lp = O.prior_draw(seed + p, 0, n)
        want = O.Ctx(inst).eval(s)
        err = np.abs(lnl[p] - want) / (np.maximum(1.0, np.abs(want)) if rel else 1.0)
        assert np.all(np.isfinite(lnl[p]))
        assert err.max() <= tol, (p, inst.n_lm, inst.n_t, err.max())
        ref = O.integrate(want, lp, lp)
        assert abs(res[p]["ln_L_marg"] - ref["ln_L_marg"]) <= (1e-9 if not rel else 1e-3)
        assert res[p]["n_samples"] == n
    return res


@pytest.mark.parametrize("precision,tol,rel", [("fp64", 1e-9, False), ("fp32", 1e-4, True),
                                               ("bf16", 1e-4, True)])
def test_batch_matches_oracle(torch, points, precision, tol, rel):
    with ile.Batch(precision) as b:
        for inst in points:
            b.add_point(inst)
        assert b.n_points == len(points)
        _check_batch(b, points, 500, 2003, tol, rel)
        # other tunings give the same answers: the pipelined engine (the
        # only BF16 one, which takes at most 256 positions per block in a
        # batch), one workgroup per CU, queue in point order
        b.set_tuning(threads=256 if precision == "bf16" else 512, wgs_per_cu=1, order=1,
                     engine=2)
        _check_batch(b, points, 501, 2003, tol, rel)


def test_batch_bf16_widest_pipelined_block_refused(torch, points):
    with ile.Batch("bf16") as b:
        b.add_point(points[0])
        with pytest.raises(ile.IleError):
            b.set_tuning(threads=512, wgs_per_cu=1, order=0, engine=2)


def test_batch_graph_replay_deterministic(torch, points):
    with ile.Batch("fp32") as b:
        for inst in points[:4]:
            b.add_point(inst)
        r1 = b.run(7, 4000)
        l1 = b.lnL(4000)
        r2 = b.run(8, 4000)
        r3 = b.run(7, 4000)
        l3 = b.lnL(4000)
    assert r1 == r3 and np.array_equal(l1, l3)
    assert r1 != r2


def test_batch_autotune_and_cache(torch, points, tmp_path):
    cache = str(tmp_path / "tune.txt")
    with ile.Batch("fp32") as b:
        for inst in points[:3]:
            b.add_point(inst)
        t = b.autotune(1000, cache)
        assert t["threads"] in (128, 192, 256, 512) and 1 <= t["wgs_per_cu"] <= 3
        assert t["engine"] in (0, 1, 2)
        lines = open(cache).read().splitlines()
        assert len(lines) == 1 and lines[0].split()[1] == str(t["threads"])
        _check_batch(b, points[:3], 42, 1000, 1e-4, True)
    with ile.Batch("fp32") as b2:
        for inst in points[:3]:
            b2.add_point(inst)
        assert b2.autotune(1000, cache) == t            # read from the cache
        assert len(open(cache).read().splitlines()) == 1


def test_batch_full_size_sampled(torch):
    """The batched workload at full size in the benchmark's launch
    configuration (256 points, Q 16384 points in FP32, 2e5 prior samples per
    point, default tuning): 64 sampled samples of every 16th point against
    the FP64 oracle (1e-4 relative, the FP32 bar), and ln L_marg of three
    points against the oracle's reduction of all their samples (1e-3)."""
    from oracle import oracle as O
    pts = [synth.batched_point(p) for p in range(256)]
    n, seed = 200_000, 11
    with ile.Batch("fp32") as b:
        for inst in pts:
            b.add_point(inst)
        res = b.run(seed, n)
        lnl = b.lnL(n)
    rng = np.random.default_rng(5)
    worst = 0.0
    for p in range(0, 256, 16):
        s, lp = O.prior_draw(seed + p, 0, n)
        idx = rng.choice(n, 64, replace=False)
        want = O.Ctx(pts[p]).eval(s[:, idx])
        err = np.abs(lnl[p][idx] - want) / np.maximum(1.0, np.abs(want))
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-4, (p, pts[p].n_lm, pts[p].n_t, err.max())
    for p in (0, 100, 255):
        s, lp = O.prior_draw(seed + p, 0, n)
        ref = O.integrate(O.Ctx(pts[p]).eval(s), lp, lp)
        assert abs(res[p]["ln_L_marg"] - ref["ln_L_marg"]) <= 1e-3
    print(f"batched full size: sampled max rel err {worst:.2e}")


def test_batch_items_beyond_one_dispatch(torch):
    """More (point, tile) items than one dispatch takes (2^22 of 512
    work-items each: 68 points x 1e6 draws are 4.25e6 items): every point's
    result equals the same point evaluated alone on the same draws, bit for
    bit, including the points of the second dispatch."""
    n, P = 1_000_000, 68
    base = synth.make_instance(["D1", "D2"], 5, 4096, 4096.0, 201, 8101)
    print(f"items beyond one dispatch: {P} points x {n}", flush=True)
    X = torch.empty((P, 7, n), dtype=torch.float64, device="cuda")
    with ile.Context(base, precision="fp32") as c:
        for p in range(P):
            c.draw_prior_dev(8200 + p, 0, n, X[p], n)
        c.sync()
    with ile.Batch("fp32") as b:
        for _ in range(P):
            b.add_point(base)
        allp = b.run_dev(n, X)
    assert all(np.isfinite(r["ln_L_marg"]) and r["n_samples"] == n for r in allp)
    for p in (0, P - 1):
        with ile.Batch("fp32") as b1:
            b1.add_point(base)
            one = b1.run_dev(n, X[p:p + 1].contiguous())[0]
        assert one["ln_L_marg"] == allp[p]["ln_L_marg"] and one["n_eff"] == allp[p]["n_eff"]
