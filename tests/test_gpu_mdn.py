"""GPU parity of the learned proposal (ile_prop_*) against the FP64 oracle.

Tolerances.  The device network runs layers 2 and 3 with BF16 operands
(unit roundoff 2^-9) and FP32 accumulation, so its ln q differs from the
FP64 oracle by the effect of those roundings.  The test measures that effect
per sample by evaluating the oracle's weights with the same roundings on
the CPU (h1, h2 and W2, W3 rounded to BF16 to nearest even, FP32 sums) and
accepts |gpu - oracle| <= 2 |bf16 emulation - oracle| + 1e-3 max(1, |ln q|).
Gradients (P11, device side): per tensor, cosine similarity >= 0.999 and
relative norm of the difference <= 1e-2.  Sampler (P12): the ln q returned
with each draw equals ile_prop_logpdf_dev's bit for bit; each dimension's
conditional CDF at the draws is uniform (probability integral transform,
Kolmogorov-Smirnov); draws from the defensive mixture integrate the prior
to 1 (E_q[p/q] = 1 within 4 standard errors).
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

from paper_1902_04934_amd import ile, synth

pytestmark = pytest.mark.gpu

OFF = dict(W1=(0, 896), b1=(896, 1024), W2=(1024, 17408), b2=(17408, 17536),
           W3=(17536, 60544), b3=(60544, 60880))


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def _bf16(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _emulated_lnq(O, P, tr, x):
    """ln q with the device's roundings (BF16 layer-2/3 operands, FP32 sums)."""
    m = O.mdn_mask().astype(np.float64)
    Pm = P * m
    W1 = Pm[0:896].reshape(128, 7).astype(np.float32)
    b1 = Pm[896:1024].astype(np.float32)
    W2 = _bf16(Pm[1024:17408].reshape(128, 128))
    b2 = Pm[17408:17536].astype(np.float32)
    W3 = _bf16(Pm[17536:60544].reshape(336, 128))
    b3 = Pm[60544:].astype(np.float32)
    n = x.shape[1]
    out = np.empty(n)
    for i in range(n):
        z, lj = O.mdn_to_z(tr, x[:, i])
        zf = z.astype(np.float32)
        h1 = _bf16(np.tanh(W1 @ zf + b1))
        h2 = _bf16(np.tanh((W2 @ h1).astype(np.float32) + b2))
        o = ((W3 @ h2).astype(np.float32) + b3).astype(np.float64)
        tot = 0.0
        for d in range(7):
            al, mu, rho = o[48 * d:48 * d + 16], o[48 * d + 16:48 * d + 32], o[48 * d + 32:48 * d + 48]
            sig = tr.sigma_scale * (tr.sigma_floor + np.logaddexp(0.0, rho))
            tot += logsumexp(al - logsumexp(al) + stats.norm.logpdf(zf[d], mu, sig))
        out[i] = tot + lj
    return out


def _transform():
    return dict(origin=[1.0, 0.5, 4.0], mean=[0.1, -0.2, 0.3, 0.0, 0.5, -1.0, 0.2],
                scale=[1.5, 0.7, 1.0, 2.0, 0.9, 1.1, 0.8])


def _prop(inst=None, seed=3, kappa=1.0):
    return ile.Proposal(seed=seed, sigma_scale=kappa)


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (64, 1.0), (1000, 1.0), (4099, 1.0), (1000, 1.25)])
def test_logpdf_matches_oracle(torch, n, kappa):
    from oracle import oracle as O
    P = synth.mdn_params(21, gain=1.0)
    T = _transform()
    tr = O.mdn_transform(**T, sigma_scale=kappa)
    x, _ = synth.prior_samples(n, 500 + n)
    want = O.mdn_logpdf(P.astype(np.float64), tr, x)
    emu = _emulated_lnq(O, P.astype(np.float64), tr, x[:, :min(n, 400)])
    with _prop(kappa=kappa) as p:
        p.set_params(P)
        p.set_transform(**T)
        xd = torch.from_numpy(x).cuda()
        lq = torch.zeros(n, dtype=torch.float64, device="cuda")
        p.logpdf_dev(xd, n, n, lq)
        p.sync()
        got = lq.cpu().numpy()
    k = emu.size
    tol = 2 * np.abs(emu - want[:k]) + 1e-3 * np.maximum(1.0, np.abs(want[:k]))
    err = np.abs(got[:k] - want[:k])
    print(f"n={n} max|gpu-orc|={err.max():.3e} max|emu-orc|={np.abs(emu - want[:k]).max():.3e} "
          f"max|gpu-emu|={np.abs(got[:k] - emu).max():.3e}")
    assert np.all(err <= tol)
    rel = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    assert rel.max() < 2e-2


def test_gradient_matches_oracle(torch):
    from oracle import oracle as O
    P = synth.mdn_params(22, gain=1.2).astype(np.float64)
    T = _transform()
    tr = O.mdn_transform(**T)
    n = 1000
    x, _ = synth.prior_samples(n, 601)
    w = np.random.default_rng(5).uniform(0.05, 2.0, n)
    loss_o, g_o = O.mdn_loss_grad(P, tr, x, w)
    # the proposal's sigma scale does not enter training
    with _prop(kappa=1.3) as p:
        p.set_params(P.astype(np.float32))
        p.set_transform(**T)
        xd = torch.from_numpy(x).cuda()
        wd = torch.from_numpy(w).cuda()
        gd = torch.zeros(O.MDN_NPARAM, dtype=torch.float32, device="cuda")
        loss_g = p.grad_dev(xd, n, n, wd, gd)
        g = gd.cpu().numpy().astype(np.float64)
    assert abs(loss_g - loss_o) <= 1e-3 * abs(loss_o), (loss_g, loss_o)
    mask = O.mdn_mask()
    assert np.all(g[mask == 0] == 0.0)
    for name, (lo, hi) in OFF.items():
        a, b = g[lo:hi], g_o[lo:hi]
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        print(f"{name}: cos={cos:.6f} rel={rel:.3e}")
        assert cos >= 0.999 and rel <= 1e-2, name


def test_fit_transform_matches_oracle(torch):
    from oracle import oracle as O
    n = 30_000
    x, _ = synth.prior_samples(n, 602)
    rng = np.random.default_rng(6)
    x[0] = np.mod(rng.vonmises(0.3, 3.0, n), 2 * np.pi)
    lnw = rng.normal(0, 4.0, n)   # tempered: the effective size of e^lnw is below 1%
    lnw[5] = -np.inf
    assert O.mdn_tempering(lnw, 0.01)[0] < 1.0
    want = O.mdn_fit_transform(x, lnw, ess_frac=0.01)
    with _prop() as p:
        p.fit_transform_dev(torch.from_numpy(x).cuda(), n, torch.from_numpy(lnw).cuda(), n, 0.01)
        o, m, s = p.get_transform()
    assert np.allclose(o, list(want.origin), rtol=0, atol=1e-10)
    assert np.allclose(m, list(want.mean), rtol=1e-10, atol=1e-12)
    assert np.allclose(s, list(want.scale), rtol=1e-10, atol=1e-12)


def _sample(torch, p, seed, first, n, eps=0.0):
    xd = torch.zeros((7, n), dtype=torch.float64, device="cuda")
    lp = torch.zeros(n, dtype=torch.float64, device="cuda")
    lq = torch.zeros(n, dtype=torch.float64, device="cuda")
    p.sample_dev(seed, first, n, xd, n, lp, lq, eps=eps)
    return xd, lp, lq


@pytest.mark.parametrize("eps,kappa", [(0.0, 1.0), (0.1, 1.0), (0.1, 1.25)])
def test_sample_lnq_is_logpdf_bitwise(torch, eps, kappa):
    """P12 (device): ln q of each draw equals logpdf of the drawn sample."""
    inst = synth.config1()
    n = 20_011
    with ile.Context(inst) as ctx:
        rng = np.random.default_rng(7)
        P_ra = rng.gamma(1.5, size=50)
        P_sd = rng.gamma(1.5, size=50)
        ile.ile_hist_set(ctx.h, P_ra / P_ra.sum(), P_sd / P_sd.sum())
        with ile.Proposal(ctx, seed=4, sigma_scale=kappa) as p:
            p.set_params(synth.mdn_params(23, gain=0.8))
            p.set_transform(**_transform())
            xd, lp, lq = _sample(torch, p, 99, 1000, n, eps)
            lq2 = torch.zeros(n, dtype=torch.float64, device="cuda")
            p.logpdf_dev(xd, n, n, lq2, eps=eps)
            p.sync()
            a, b = lq.cpu().numpy(), lq2.cpu().numpy()
            x = xd.cpu().numpy()
            # a second draw of the same counters is identical
            xd3, _, lq3 = _sample(torch, p, 99, 1000, n, eps)
            p.sync()
            assert np.array_equal(xd3.cpu().numpy(), x) and np.array_equal(lq3.cpu().numpy(), a)
    assert np.all(np.isfinite(a))
    assert np.array_equal(a, b)
    # samples lie in the prior's support
    assert np.all((x[0] >= 0) & (x[0] <= 2 * np.pi)) and np.all(np.abs(x[1]) <= np.pi / 2)
    assert np.all((x[2] >= 0) & (x[2] <= np.pi)) and np.all((x[3] >= 0) & (x[3] <= 2 * np.pi))
    assert np.all(np.abs(x[4]) <= 1) and np.all((x[5] >= 10) & (x[5] <= 1000))
    assert np.all(np.abs(x[6]) <= 0.01)


@pytest.mark.parametrize("kappa", [1.0, 1.25])
def test_draws_follow_the_conditionals(torch, kappa):
    """Probability integral transform: for draws of the network alone, each
    dimension's conditional CDF (mixture from the oracle's outputs at the
    draw's earlier dimensions, sigmas widened by kappa) evaluated at the
    draw is uniform (KS)."""
    from oracle import oracle as O
    P = synth.mdn_params(26, gain=0.9)
    T = _transform()
    tr = O.mdn_transform(**T)
    n = 20_000
    with _prop(kappa=kappa) as p:
        p.set_params(P)
        p.set_transform(**T)
        xd, _, _ = _sample(torch, p, 17, 5, n)
        p.sync()
        x = xd.cpu().numpy()
    z, o = O.mdn_outputs(P.astype(np.float64), tr, x)
    for d in range(7):
        al, mu, rho = o[:, 48 * d:48 * d + 16], o[:, 48 * d + 16:48 * d + 32], o[:, 48 * d + 32:48 * d + 48]
        sig = kappa * (1e-3 + np.logaddexp(0.0, rho))
        w = np.exp(al - logsumexp(al, axis=1, keepdims=True))
        u = np.sum(w * stats.norm.cdf((z[:, d:d + 1] - mu) / sig), axis=1)
        ks = stats.kstest(u, "uniform")
        print(f"dim {d}: KS {ks.statistic:.4f} p {ks.pvalue:.3g}")
        assert ks.pvalue > 1e-4, d


@pytest.mark.parametrize("eps,kappa", [(0.25, 1.0), (0.25, 1.25)])
def test_draws_integrate_prior(torch, eps, kappa):
    """E_q[p/q] = 1 for the defensive mixture (p/q is bounded there): the
    draws follow the density their ln q describes."""
    inst = synth.config1()
    n = 400_000
    with ile.Context(inst) as ctx:
        rng = np.random.default_rng(8)
        P_ra = rng.gamma(2.0, size=40)
        P_sd = rng.gamma(2.0, size=40)
        ile.ile_hist_set(ctx.h, P_ra / P_ra.sum(), P_sd / P_sd.sum())
        with ile.Proposal(ctx, seed=5, sigma_scale=kappa) as p:
            p.set_params(synth.mdn_params(24, gain=0.6))
            p.set_transform(origin=[2.0, 1.0, 3.0], mean=[0.0] * 7, scale=[1.0] * 7)
            xd, lp, lq = _sample(torch, p, 123, 0, n, eps)
            p.sync()
            r = np.exp(lp.cpu().numpy() - lq.cpu().numpy())
    m, se = r.mean(), r.std() / math.sqrt(n)
    print(f"eps={eps}: E[p/q]={m:.5f} +- {se:.5f}")
    assert abs(m - 1.0) < 4 * se and se < 0.05


def test_sigma_scale_keeps_fitted_transform(torch):
    """Setting kappa after a device fit keeps the fitted transform; kappa
    must be positive."""
    n = 5000
    x, _ = synth.prior_samples(n, 604)
    lnw = np.random.default_rng(9).normal(0, 1.0, n)
    with _prop() as p:
        p.fit_transform_dev(torch.from_numpy(x).cuda(), n, torch.from_numpy(lnw).cuda(), n)
        before = p.get_transform()
        p.set_sigma_scale(1.3)
        after = p.get_transform()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
        with pytest.raises(ile.IleError):
            p.set_sigma_scale(0.0)


def test_first_dimension_marginal(torch):
    """Dimension 0 has no parents: its draws follow the mixture given by b3."""
    from oracle import oracle as O
    P = synth.mdn_params(25, gain=1.0)
    n = 50_000
    T = dict(origin=[1.0, 0.5, 4.0], mean=[0.2] + [0.0] * 6, scale=[1.3] + [1.0] * 6)
    tr = O.mdn_transform(**T)
    with _prop() as p:
        p.set_params(P)
        p.set_transform(**T)
        xd, _, _ = _sample(torch, p, 7, 0, n)
        p.sync()
        x = xd.cpu().numpy()
    u0 = np.mod((x[0] - 1.0) / (2 * np.pi) + 0.5, 1.0)
    z0 = (np.log(u0) - np.log1p(-u0) - 0.2) / 1.3
    b3 = P[60544:60544 + 48].astype(np.float64)
    al, mu, rho = b3[:16], b3[16:32], b3[32:48]
    sig = 1e-3 + np.logaddexp(0.0, rho)
    wts = np.exp(al - logsumexp(al))
    cdf = lambda z: np.sum(wts[None, :] * stats.norm.cdf((np.asarray(z)[:, None] - mu) / sig), axis=1)
    ks = stats.kstest(z0, cdf)
    print("KS", ks)
    assert ks.pvalue > 1e-3


def test_training_is_reproducible_and_learns(torch):
    """Training on weighted samples lowers the loss, and two runs with the
    same seeds give bit-identical weights."""
    n = 60_000
    x, _ = synth.prior_samples(n, 603)
    # a target concentrated in ra, dec and cos iota
    lnw = (-0.5 * ((x[0] - 2.0) / 0.3) ** 2 - 0.5 * ((np.sin(x[1]) - 0.4) / 0.2) ** 2
           - 0.5 * ((x[4] - 0.7) / 0.2) ** 2)
    xd = torch.from_numpy(x).cuda()
    wd = torch.from_numpy(lnw).cuda()
    out = []
    for _ in range(2):
        with _prop(seed=9) as p:
            l0 = None
            p.fit_transform_dev(xd, n, wd, n, 0.01)
            # loss before training, on the tempered weights
            from oracle import oracle as O
            beta = O.mdn_tempering(lnw, 0.01)[0]
            w = torch.from_numpy(np.exp(beta * (lnw - lnw.max()))).cuda()
            l0 = p.grad_dev(xd, n, 4096, w)
            l1 = p.train_dev(xd, n, wd, n, steps=300, batch=2048, lr=2e-3, seed=11,
                             fit_transform=False)
            l2 = p.grad_dev(xd, n, 4096, w)
            out.append((p.get_params(), l0, l1, l2, p.last_ms()))
    (pa, l0, l1, l2, ms), (pb, *_rest) = out
    print(f"loss {l0:.4f} -> {l2:.4f} (last minibatch {l1:.4f}); {ms:.1f} ms for 300 steps")
    assert np.array_equal(pa, pb)
    assert l2 < l0 - 0.5
