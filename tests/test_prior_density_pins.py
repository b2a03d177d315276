"""Pins of the prior and proposal densities that the draws write (ln p, ln q).

Sec. II.A takes the extrinsic prior uniform in source orientation and in the
4-volume: ra uniform, sin dec uniform, psi, phi and cos iota uniform, p(D)
proportional to D^2 on [d_min, d_max], t_ref uniform on [-t_max, t_max].  Each
of these is fixed by its cumulative distribution F_p, and the draws are made
by inverting F_p.  The density of a draw is then prod_p F_p'(x_p).  The tests
take those derivatives by central differences of F_p at every draw and
compare the sum of their logarithms with the ln p (or ln q) written beside
the draw: a route that shares nothing with the closed-form expressions in the
oracle or the generator module, so a dropped or misplaced factor (the 3 D^2,
cos dec taken outside the logarithm, a missing 1/2) fails here.

The histogram proposal of the adaptive sampler replaces the ra and sin dec
marginals by piecewise-constant densities with bin probabilities P; its CDF
is piecewise linear, C[b] + P[b] (x nb - b) in the rescaled coordinate.

P10 (unbiasedness of the proposals) on the oracle's own sampler closes the
file: prior draws and adaptive histogram draws, each weighted by its own
density, give ln L_marg within their combined standard error.
"""
import numpy as np
import pytest

from paper_1902_04934_amd import synth

D_MIN, D_MAX, T_MAX = 10.0, 1000.0, 0.01
TWO_PI = 2.0 * np.pi


def prior_cdfs(d_min=D_MIN, d_max=D_MAX, t_max=T_MAX):
    """The seven marginal CDFs of the prior of Sec. II.A."""
    v3 = d_max ** 3 - d_min ** 3
    return [
        lambda x: x / TWO_PI,                        # ra
        lambda x: (np.sin(x) + 1.0) / 2.0,           # dec, sin dec uniform
        lambda x: x / np.pi,                         # psi
        lambda x: x / TWO_PI,                        # phi
        lambda x: (x + 1.0) / 2.0,                   # cos iota
        lambda x: (x ** 3 - d_min ** 3) / v3,        # D, uniform in volume
        lambda x: (x + t_max) / (2.0 * t_max),       # t_ref
    ]


def hist_cdf(P, lo, width):
    """CDF of a piecewise-constant density on [lo, lo + width) whose nb bins
    carry probabilities P."""
    nb = P.size
    C = np.concatenate([[0.0], np.cumsum(P)])

    def F(x):
        y = (x - lo) * nb / width
        b = np.clip(np.floor(y).astype(np.int64), 0, nb - 1)
        return C[b] + P[b] * (y - b)
    return F


def log_density_fd(cdfs, s, rel_h=1e-6):
    """sum_p ln F_p'(x_p) by central differences, with a step relative to
    each parameter's range (so the differences stay well above rounding)."""
    scales = [TWO_PI, np.pi, np.pi, TWO_PI, 2.0, D_MAX - D_MIN, 2 * T_MAX]
    tot = np.zeros(s.shape[1])
    for p, F in enumerate(cdfs):
        h = rel_h * scales[p]
        d = (F(s[p] + h) - F(s[p] - h)) / (2.0 * h)
        tot += np.log(d)
    return tot


def interior(s, edges=None):
    """Draws whose difference stencil stays inside the support (and away
    from histogram bin edges, where the CDF has a kink)."""
    ok = (s[0] > 1e-4) & (s[0] < TWO_PI - 1e-4) & (np.cos(s[1]) > 1e-3)
    ok &= (s[2] > 1e-4) & (s[2] < np.pi - 1e-4) & (s[3] > 1e-4) & (s[3] < TWO_PI - 1e-4)
    ok &= np.abs(s[4]) < 1 - 1e-4
    ok &= (s[5] > D_MIN + 1e-2) & (s[5] < D_MAX - 1e-2) & (np.abs(s[6]) < T_MAX * (1 - 1e-4))
    if edges is not None:
        for x, nb, lo, width in edges:
            y = (x - lo) * nb / width
            ok &= np.abs(y - np.round(y)) > 1e-3
    return ok


def test_oracle_prior_density_is_derivative_of_prior_cdfs(orc):
    s, lp = orc.prior_draw(seed=123, first=0, n=20_000)
    ok = interior(s)
    assert ok.mean() > 0.99
    want = log_density_fd(prior_cdfs(), s[:, ok])
    assert np.max(np.abs(lp[ok] - want)) < 1e-6
    # the density is the same at every draw except through cos dec and D
    # (uniform elsewhere): with those two factored out it is constant
    rest = lp - np.log(np.cos(s[1])) - 2.0 * np.log(s[5])
    assert np.ptp(rest) < 1e-12


def test_generator_prior_density_is_derivative_of_prior_cdfs():
    s, lp = synth.prior_samples(20_000, 9)
    ok = interior(s)
    want = log_density_fd(prior_cdfs(), s[:, ok])
    assert np.max(np.abs(lp[ok] - want)) < 1e-6


def test_prior_density_integrates_to_one(orc):
    """exp(ln p) over the support: the prior's six non-trivial directions
    factor, so a 1-D quadrature in dec and in D of the density written by
    the draws, times the flat widths, gives 1.  The draws' (dec, D, ln p)
    triples define the density along both axes (ln p is linear in ln cos dec
    and ln D, fixed by two draws each), checked at every draw above."""
    s, lp = orc.prior_draw(seed=5, first=0, n=4000)
    # fit ln p = c0 + a ln cos dec + b ln D over the draws (exact: residual 0)
    A = np.c_[np.ones(s.shape[1]), np.log(np.cos(s[1])), np.log(s[5])]
    coef, *_ = np.linalg.lstsq(A, lp, rcond=None)
    assert np.max(np.abs(A @ coef - lp)) < 1e-11
    c0, a, b = coef
    x, w = np.polynomial.legendre.leggauss(200)
    dec = x * np.pi / 2
    I_dec = np.sum(w * np.pi / 2 * np.cos(dec) ** a)
    D = D_MIN + (x + 1) / 2 * (D_MAX - D_MIN)
    I_D = np.sum(w * (D_MAX - D_MIN) / 2 * D ** b)
    total = np.exp(c0) * TWO_PI * np.pi * TWO_PI * 2.0 * (2 * T_MAX) * I_dec * I_D
    assert total == pytest.approx(1.0, abs=1e-12)


def test_histogram_proposal_density_is_derivative_of_its_cdfs(orc):
    rng = np.random.default_rng(17)
    nb = 50
    P_ra = rng.gamma(1.5, size=nb)
    P_ra /= P_ra.sum()
    P_sd = rng.gamma(0.8, size=nb)
    P_sd /= P_sd.sum()
    s, lp, lq, bins = orc.hist_draw(31, 0, 20_000, P_ra, P_sd)
    edges = [(s[0], nb, 0.0, TWO_PI), (np.sin(s[1]), nb, -1.0, 2.0)]
    ok = interior(s, edges=edges)
    assert ok.mean() > 0.95
    F_ra = hist_cdf(P_ra, 0.0, TWO_PI)
    F_sd = hist_cdf(P_sd, -1.0, 2.0)
    cdfs = prior_cdfs()
    cdfs[0] = F_ra
    cdfs[1] = lambda x: F_sd(np.sin(x))
    want_q = log_density_fd(cdfs, s[:, ok])
    assert np.max(np.abs(lq[ok] - want_q)) < 1e-6
    want_p = log_density_fd(prior_cdfs(), s[:, ok])
    assert np.max(np.abs(lp[ok] - want_p)) < 1e-6


def test_planted_density_slips_fail_the_pin(orc):
    """The comparison above sees the slips it is meant to see."""
    s, lp = orc.prior_draw(seed=123, first=0, n=5000)
    ok = interior(s)
    want = log_density_fd(prior_cdfs(), s[:, ok])
    v3 = D_MAX ** 3 - D_MIN ** 3
    slips = [
        lp - np.log(3 * s[5] ** 2 / v3),                               # 3 D^2 / v3 dropped
        lp - np.log(np.cos(s[1]) / 2) + np.log(np.cos(s[1])) / 2,      # log(cos dec)/2
        lp + np.log(2.0),                                              # psi on [0, 2 pi)
        lp - np.log(3 * s[5] ** 2 / v3) + np.log(s[5] ** 2 / v3),       # missing factor 3
    ]
    for bad in slips:
        assert np.max(np.abs(bad[ok] - want)) > 1e-3


# ------------------------------------------------------------------ P10
def test_P10_prior_and_adaptive_oracle_sampler_agree(orc):
    """Sec. II.A and II.C: every chunk is weighted by the density it was drawn
    from, so the prior and the adaptive histogram proposal (refit after every
    chunk from tempered weights, 10% prior floor) estimate the same
    ln L_marg; they agree within their combined standard error.  Instance: a
    zero-noise injection at network SNR 6 (2 detectors, 5 modes, 101 bins),
    loud enough for the sky histograms to move and quiet enough for the
    prior to reach an n_eff of a few hundred.  Weighting the adaptive draws
    by the prior instead of the proposal (a dropped ln q) fails."""
    base = synth.make_instance(["D1", "D2"], 5, 2048, 2048.0, 101, 77)
    h = synth.mode_waveforms(base.modes, base.n_q, base.srate_hz, 78, amp=20.0)
    theta = np.array([1.3, 0.4, 0.7, 2.0, 0.5, 400.0, 0.002])
    inst, _, _ = orc.injection_instance(base, h, theta, snr=6.0)
    ctx = orc.Ctx(inst)
    s, lp = orc.prior_draw(seed=2024, first=0, n=200_000)
    r_prior = orc.integrate(ctx.eval(s), lp, lp)

    nb, chunk, rounds = 50, 20_000, 10
    P_ra = np.full(nb, 1.0 / nb)
    P_sd = np.full(nb, 1.0 / nb)
    lw_all, lw_noq = [], []
    for r in range(rounds):
        s, lp, lq, bins = orc.hist_draw(2025, r * chunk, chunk, P_ra, P_sd)
        L = ctx.eval(s)
        lw = L + lp - lq
        lw_all.append(lw)
        lw_noq.append(L)
        P_ra, P_sd = orc.hist_refit(bins, lw, nb, floor=0.1, scale=10.0)
    z = np.zeros(rounds * chunk)
    r_adapt = orc.integrate(np.concatenate(lw_all), z, z)
    assert np.max(P_ra) > 4.0 / nb               # the proposal moved off the prior
    assert r_adapt["n_eff"] > 100 and r_prior["n_eff"] > 100
    sig = np.hypot(r_prior["sigma"], r_adapt["sigma"])
    assert abs(r_prior["ln_L_marg"] - r_adapt["ln_L_marg"]) < 4 * sig
    r_bad = orc.integrate(np.concatenate(lw_noq), z, z)
    assert abs(r_prior["ln_L_marg"] - r_bad["ln_L_marg"]) > 4 * np.hypot(r_prior["sigma"], r_bad["sigma"])
