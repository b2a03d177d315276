"""Proposal reuse across intrinsic points (the integrator reused for each
lambda, Sec. II.C): learned runs over a sequence of neighbouring points
(synth.lambda_sequence: the learned-proposal workload with the stand-in
chirp's intrinsic parameters stepped by 1% per point), cold (every point from
scratch) and warm (network and histograms carried from point to point,
ile_run with warm = 1).

* Cold and warm estimates of every point agree within 4 combined standard
  errors: each is unbiased whatever proposal it used.
* No warm run falls back, and each reaches the n_eff target; after the
  first point the warm sequence spends fewer refits than the cold one (the
  paper's faster convergence from reuse).
* Same samples, same weights: a chunk of the last warm mixture evaluated on
  the device gives the oracle's ln L_marg within 1e-3.
"""
import numpy as np
import pytest

from paper_1902_04934_amd import ile, reuse, synth

pytestmark = pytest.mark.gpu

TARGET = 1e4


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def runs(torch):
    pts = synth.lambda_sequence(5)
    cold = reuse.run(pts, warm=False, target=TARGET)
    warm = reuse.run(pts, warm=True, target=TARGET)
    for tag, rs in (("cold", cold), ("warm", warm)):
        for p, r in enumerate(rs):
            print(f"{tag} point {p}: {r['seconds']:.3f} s, refits {r['refits']}, "
                  f"fell_back {r['fell_back']}, n_eff {r['n_eff']:.0f}, "
                  f"ln L {r['ln_L_marg']:.5f} +- {r['sigma_ln_L']:.5f}, "
                  f"train {r['train_ms']:.1f} ms", flush=True)
    return pts, cold, warm


def test_warm_and_cold_agree(runs):
    _, cold, warm = runs
    for c, w in zip(cold, warm):
        if c["fell_back"]:
            continue
        sig = np.hypot(c["sigma_ln_L"], w["sigma_ln_L"])
        assert abs(c["ln_L_marg"] - w["ln_L_marg"]) < 4 * sig + 1e-3


def test_warm_runs_reach_target(runs):
    _, _, warm = runs
    assert not warm[0]["warm"] and all(r["warm"] for r in warm[1:])
    for r in warm:
        assert r["fell_back"] == 0
        assert r["n_eff"] >= TARGET
    cold = runs[1]
    assert sum(r["refits"] for r in warm[1:]) < sum(r["refits"] for r in cold[1:])


def test_warm_mixture_same_sample_parity(torch, runs):
    """A network trained on the last point, then a warm run on that point
    from it (its rounds drawn from the network's mixture): the run reaches
    the target without falling back, and the device ln L_marg of the
    mixture's draws equals the oracle's on the same samples and weights."""
    from oracle import oracle as O
    pts = runs[0]
    last = pts[-1]
    ctx, inst = reuse.combined.injected_point(last, "fp64")
    with ctx, ile.Proposal(ctx, seed=3) as prop:
        r = ctx.run(sampler="learned", seed=99, chunk=100_000, max_samples=100_000,
                    adapt_chunks=3, prop=prop, eps=0.1)
        assert r["fell_back"] == 0
        n = 20_000
        xd = torch.zeros((7, n), dtype=torch.float64, device="cuda")
        lp = torch.zeros(n, dtype=torch.float64, device="cuda")
        lq = torch.zeros(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        # warm start on the same point from this trained network: the rounds
        # draw from its mixture
        w = ctx.run(sampler="learned", seed=123, chunk=100_000, max_samples=2_000_000,
                    n_eff_target=TARGET, adapt_chunks=3, prop=prop, eps=0.1, reset=False,
                    warm=True)
        assert w["fell_back"] == 0 and w["n_eff"] >= TARGET
        prop.sample_dev(4243, 0, n, xd, n, lp, lq, eps=0.1)
        prop.sync()
        x, lpv, lqv = xd.cpu().numpy(), lp.cpu().numpy(), lq.cpu().numpy()
        got = ctx.integrate(x, lpv, lqv)
    lnL = O.Ctx(inst).eval(x)
    ref = O.integrate(lnL, lpv, lqv)
    print("same-sample:", got["ln_L_marg"], ref["ln_L_marg"])
    assert abs(got["ln_L_marg"] - ref["ln_L_marg"]) <= 1e-3
