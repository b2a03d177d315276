"""Pins of the oracle's learned proposal (mixture-density network).

The network is this library's own model (the paper adapts histograms only),
so what pins it is mathematics, not printed values:
  * P11: the hand-written back-propagation equals central finite
    differences of the loss (relative 1e-6);
  * P12: the density is normalized: E_prior[q/p] = 1 within 4 sigma, and
    each conditional integrates to 1 by quadrature;
  * the masks make the model autoregressive (ln q_d ignores z~_j, j >= d);
  * with W3 = 0 every conditional is the fixed mixture b3 (scipy's normal),
    with every sigma multiplied by the sigma scale kappa;
  * the training loss and gradient are those of the kappa = 1 model;
  * the transform fit gives circular means and weighted moments.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

from oracle import oracle as O
from paper_1902_04934_amd import synth

NP = O.MDN_NPARAM
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 896, 1024, 17408, 17536, 60544


def params(seed=11, gain=1.0):
    return synth.mdn_params(seed, gain=gain).astype(np.float64)


def test_layout_and_mask_counts():
    m = O.mdn_mask()
    assert m.size == NP == OFF_B3 + 336
    # W1: unit k sees inputs 0..k%6 -> sum over k of (k%6 + 1)
    assert m[OFF_W1:OFF_B1].sum() == sum((k % 6) + 1 for k in range(128))
    # W2: k2 sees k1 with k1%6 <= k2%6
    deg = np.arange(128) % 6
    assert m[OFF_W2:OFF_B2].sum() == int((deg[None, :] <= deg[:, None]).sum())
    # W3: output o (dimension o//48) sees units with degree < o//48
    assert m[OFF_W3:OFF_B3].sum() == sum(int((deg < o // 48).sum()) for o in range(336))
    assert m[OFF_B1:OFF_W2].all() and m[OFF_B2:OFF_W3].all() and m[OFF_B3:].all()


def test_autoregressive():
    P = params(3)
    tr = O.mdn_transform()
    rng = np.random.default_rng(0)
    z = rng.standard_normal(7)
    _, base = O.mdn_lnq_z(P, tr, z)
    for j in range(7):
        z2 = z.copy()
        z2[j] += 0.7
        _, d2 = O.mdn_lnq_z(P, tr, z2)
        # terms before j are unchanged exactly; term j and later change
        assert np.array_equal(d2[:j], base[:j]), j
        assert d2[j] != base[j]
        if j < 6:
            assert np.any(d2[j + 1:] != base[j + 1:])


@pytest.mark.parametrize("kappa", [1.0, 1.25])
def test_constant_outputs_reduce_to_scipy_mixture(kappa):
    P = params(4)
    P[OFF_W3:OFF_B3] = 0.0
    b3 = P[OFF_B3:]
    tr = O.mdn_transform(sigma_floor=1e-3, sigma_scale=kappa)
    z = np.array([0.3, -1.2, 0.0, 2.1, -0.4, 0.9, -2.5])
    _, dims = O.mdn_lnq_z(P, tr, z)
    for d in range(7):
        o = b3[48 * d:48 * d + 48]
        logits, mu, rho = o[:16], o[16:32], o[32:]
        sig = kappa * (1e-3 + np.logaddexp(0.0, rho))
        lw = logits - logsumexp(logits)
        ref = logsumexp(lw + stats.norm.logpdf(z[d], mu, sig))
        assert abs(dims[d] - ref) <= 1e-13 * max(1.0, abs(ref)), d


@pytest.mark.parametrize("kappa", [1.0, 1.3])
def test_conditionals_integrate_to_one(kappa):
    """For fixed earlier dimensions, each conditional density integrates to
    1 over z~_d (trapezoid on a fine grid), widened or not."""
    P = params(5, gain=1.5)
    tr = O.mdn_transform(sigma_scale=kappa)
    rng = np.random.default_rng(1)
    z = rng.standard_normal(7)
    grid = np.linspace(-30, 30, 24001)
    for d in (0, 3, 6):
        vals = np.empty(grid.size)
        for i, g in enumerate(grid):
            zz = z.copy()
            zz[d] = g
            vals[i] = O.mdn_lnq_z(P, tr, zz)[1][d]
        integral = np.trapezoid(np.exp(vals), grid)
        assert abs(integral - 1.0) < 1e-6, (d, integral)


@pytest.mark.parametrize("kappa", [1.0, 1.25])
def test_normalization_under_prior(kappa):
    """P12 (oracle side): E_prior[q/p] = 1 within 4 standard errors."""
    P = params(6, gain=0.5)
    tr = O.mdn_transform(origin=(1.0, 0.5, 4.0), sigma_scale=kappa)
    x, lp = synth.prior_samples(60_000, 77)
    lq = O.mdn_logpdf(P, tr, x)
    r = np.exp(lq - lp)
    m, se = r.mean(), r.std() / math.sqrt(r.size)
    assert abs(m - 1.0) < 4 * se and se < 0.05, (m, se)


def test_jacobian_matches_numerical_derivative():
    """ln |dz~/dx| of the transform equals the log of a central difference of
    the map x -> z~ per dimension (the map is diagonal)."""
    tr = O.mdn_transform(origin=(1.0, 0.5, 4.0), mean=[0.1, -0.2, 0.3, 0.0, 0.5, -1.0, 0.2],
                         scale=[1.5, 0.7, 1.0, 2.0, 0.9, 1.1, 0.8])
    x = np.array([2.0, 0.4, 1.3, 0.2, -0.3, 400.0, 0.004])
    z, lj = O.mdn_to_z(tr, x)
    tot = 0.0
    for d in range(7):
        h = 1e-6 * max(1.0, abs(x[d])) if d != 6 else 1e-9
        xp, xm = x.copy(), x.copy()
        xp[d] += h
        xm[d] -= h
        dz = (O.mdn_to_z(tr, xp)[0][d] - O.mdn_to_z(tr, xm)[0][d]) / (2 * h)
        tot += math.log(abs(dz))
    assert abs(tot - lj) < 1e-6


def test_boundary_gives_minus_inf():
    tr = O.mdn_transform()
    x = np.array([[1.0], [0.2], [0.3], [0.4], [-1.0], [100.0], [0.0]])   # cos iota = -1
    P = params(7)
    assert O.mdn_logpdf(P, tr, x)[0] == -np.inf


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_matches_finite_differences(weighted):
    """P11: analytic gradient vs central differences, relative 1e-6."""
    P = params(8, gain=1.2)
    tr = O.mdn_transform(origin=(0.5, 1.0, 2.0))
    x, _ = synth.prior_samples(6, 12)
    w = np.random.default_rng(2).uniform(0.1, 2.0, 6) if weighted else None
    loss, g = O.mdn_loss_grad(P, tr, x, w)
    mask = O.mdn_mask()
    assert np.all(g[mask == 0] == 0.0)
    rng = np.random.default_rng(3)
    idx = []
    for lo, hi in ((OFF_W1, OFF_B1), (OFF_B1, OFF_W2), (OFF_W2, OFF_B2), (OFF_B2, OFF_W3),
                   (OFF_W3, OFF_B3), (OFF_B3, NP)):
        cand = np.arange(lo, hi)[mask[lo:hi] == 1]
        idx.extend(rng.choice(cand, 12, replace=False))
    for j in idx:
        h = 1e-5
        Pp, Pm = P.copy(), P.copy()
        Pp[j] += h
        Pm[j] -= h
        fd = (O.mdn_loss_grad(Pp, tr, x, w)[0] - O.mdn_loss_grad(Pm, tr, x, w)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(abs(g[j]), 1e-3), (j, fd, g[j])


def test_loss_ignores_sigma_scale():
    """Training fits the kappa = 1 model: the loss and gradient do not
    depend on the sigma scale, and the loss is the kappa = 1 density's."""
    P = params(10, gain=1.1)
    x, _ = synth.prior_samples(7, 15)
    w = np.random.default_rng(6).uniform(0.2, 1.5, 7)
    l1, g1 = O.mdn_loss_grad(P, O.mdn_transform(), x, w)
    l2, g2 = O.mdn_loss_grad(P, O.mdn_transform(sigma_scale=1.4), x, w)
    assert l1 == l2 and np.array_equal(g1, g2)
    # and the widened density differs from it
    tr = O.mdn_transform(sigma_scale=1.4)
    z, _ = O.mdn_to_z(tr, x[:, 0])
    assert O.mdn_lnq_z(P, tr, z)[0] != O.mdn_lnq_z(P, O.mdn_transform(), z)[0]


def test_loss_is_weighted_mean_nll():
    P = params(9)
    tr = O.mdn_transform()
    x, _ = synth.prior_samples(5, 13)
    w = np.array([1.0, 2.0, 0.5, 0.0, 3.0])
    loss, _ = O.mdn_loss_grad(P, tr, x, w)
    lz = []
    for i in range(5):
        z, _ = O.mdn_to_z(tr, x[:, i])
        lz.append(O.mdn_lnq_z(P, tr, z)[0])
    assert abs(loss - (-(w * np.array(lz)).sum() / w.sum())) < 1e-12 * abs(loss)


def test_fit_transform_moments():
    rng = np.random.default_rng(4)
    n = 20_000
    x, _ = synth.prior_samples(n, 14)
    # concentrate ra around 0.1 (wrapping through 0), psi around 3.0, phi around 6.2
    x[0] = np.mod(rng.vonmises(0.1, 4.0, n), 2 * np.pi)
    x[2] = np.mod(rng.vonmises(3.0 * 2, 4.0, n) / 2, np.pi)
    x[3] = np.mod(rng.vonmises(6.2, 4.0, n), 2 * np.pi)
    lnw = rng.normal(0.0, 0.5, n)
    tr = O.mdn_fit_transform(x, lnw, ess_frac=0.01)
    # ln w ~ N(0, 0.5): the untempered weights already have a large effective size
    assert O.mdn_tempering(lnw, 0.01)[0] == 1.0
    w = np.exp(lnw - lnw.max())
    for j, (d, P) in enumerate(((0, 2 * np.pi), (2, np.pi), (3, 2 * np.pi))):
        a = 2 * np.pi * x[d] / P
        ref = math.atan2((w * np.sin(a)).sum(), (w * np.cos(a)).sum()) * P / (2 * np.pi)
        assert abs(tr.origin[j] - ref) < 1e-12
    assert abs(tr.origin[0] - 0.1) < 0.03 and abs(tr.origin[2] - (6.2 - 2 * np.pi)) < 0.03
    # moments of z = logit(u) with the fitted origins
    u = np.empty((7, n))
    u[0] = np.mod((x[0] - tr.origin[0]) / (2 * np.pi) + 0.5, 1.0)
    u[1] = (np.sin(x[1]) + 1) / 2
    u[2] = np.mod((x[2] - tr.origin[1]) / np.pi + 0.5, 1.0)
    u[3] = np.mod((x[3] - tr.origin[2]) / (2 * np.pi) + 0.5, 1.0)
    u[4] = (x[4] + 1) / 2
    u[5] = (x[5] - 10.0) / 990.0
    u[6] = (x[6] + 0.01) / 0.02
    z = np.log(u) - np.log1p(-u)
    for d in range(7):
        m = np.average(z[d], weights=w)
        s = math.sqrt(np.average((z[d] - m) ** 2, weights=w))
        assert abs(tr.mean[d] - m) < 1e-9 and abs(tr.scale[d] - s) < 1e-9, d


def _kish(lnw, beta):
    w = np.exp(beta * (lnw - lnw.max()))
    return w.sum() ** 2 / (w * w).sum()


@pytest.mark.parametrize("spread", [5.0, 60.0, 400.0])
def test_tempering_reaches_target_effective_size(spread):
    """beta is the largest tempering (to 2^-30) whose Kish effective size
    reaches ess_frac of the samples; the fit uses exactly those weights."""
    rng = np.random.default_rng(int(spread))
    n = 5000
    lnw = rng.normal(0.0, spread, n)
    frac = 0.02
    beta, m = O.mdn_tempering(lnw, frac)
    assert m == lnw.max()
    target = frac * n
    if beta < 1.0:
        assert _kish(lnw, beta) >= target * (1 - 1e-12)
        assert _kish(lnw, beta + 2.0 ** -29) < target
    else:
        assert _kish(lnw, 1.0) >= target
    # larger spreads need stronger tempering
    assert (beta < 1.0) == (_kish(lnw, 1.0) < target)
    x, _ = synth.prior_samples(n, 16)
    tr = O.mdn_fit_transform(x, lnw, ess_frac=frac)
    w = np.exp(beta * (lnw - lnw.max()))
    u4 = (x[4] + 1) / 2
    z4 = np.log(u4) - np.log1p(-u4)
    assert abs(tr.mean[4] - np.average(z4, weights=w)) < 1e-9


def test_tempering_ignores_non_finite():
    lnw = np.array([0.0, -np.inf, 1.0, np.nan, 2.0])
    beta, m = O.mdn_tempering(lnw, 0.5)
    assert m == 2.0
    # the same as the finite values alone (the target counts finite values)
    assert beta == O.mdn_tempering(np.array([0.0, 1.0, 2.0]), 0.5)[0]
