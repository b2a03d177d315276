"""Pins of the oracle's plain adaptive sampler (histogram proposal in ra and
sin dec): inverse-CDF draws follow the bin probabilities, the proposal
density is normalized (E_q[p/q] = 1), a uniform histogram is the prior, and
refits equal weighted bin counts computed by numpy."""
import numpy as np
import pytest
from scipy import stats


def test_uniform_histogram_is_the_prior(orc):
    nb = 50
    P = np.full(nb, 1.0 / nb)
    s, lp, lq, bins = orc.hist_draw(5, 0, 20_000, P, P)
    sp, lpp = orc.prior_draw(5, 0, 20_000)
    for p in (2, 3, 4, 5, 6):
        assert np.array_equal(s[p], sp[p])
    assert np.max(np.abs(s[0] - sp[0])) < 1e-12
    assert np.max(np.abs(s[1] - sp[1])) < 1e-9
    assert np.max(np.abs(lq - lp)) < 1e-12


def test_draws_follow_bin_probabilities(orc):
    rng = np.random.default_rng(3)
    nb = 20
    P_ra = rng.gamma(2.0, size=nb); P_ra /= P_ra.sum()
    P_sd = rng.gamma(0.7, size=nb); P_sd /= P_sd.sum()
    n = 200_000
    s, lp, lq, bins = orc.hist_draw(11, 7, n, P_ra, P_sd)
    for b, P in ((bins[0], P_ra), (bins[1], P_sd)):
        cnt = np.bincount(b, minlength=nb)
        assert stats.chisquare(cnt, P * n).pvalue > 1e-4
    # the bin of each sample is where its coordinate lies
    assert np.array_equal(np.floor(s[0] / (2 * np.pi / nb)).astype(int).clip(0, nb - 1), bins[0])
    sd = np.sin(s[1])
    inner = np.abs((sd + 1) / (2.0 / nb) - np.round((sd + 1) / (2.0 / nb))) > 1e-9
    assert np.array_equal(np.floor((sd[inner] + 1) / (2.0 / nb)).astype(int).clip(0, nb - 1),
                          bins[1][inner])
    # normalization: E_q[p / q] = 1
    r = np.exp(lp - lq)
    assert abs(r.mean() - 1) < 4 * r.std() / np.sqrt(n)


def test_refit_is_weighted_bin_count(orc):
    rng = np.random.default_rng(4)
    nb, n = 30, 5000
    bins = np.stack([rng.integers(0, nb, n), rng.integers(0, nb, n)]).astype(np.int32)
    lnw = rng.normal(0, 1.0, n)                       # spread < scale: beta = 1
    P_ra, P_sd = orc.hist_refit(bins, lnw, nb, floor=0.0, scale=1e9)
    w = np.exp(lnw - lnw.max())
    assert np.allclose(P_ra, np.bincount(bins[0], w, nb) / w.sum(), rtol=1e-13, atol=0)
    assert np.allclose(P_sd, np.bincount(bins[1], w, nb) / w.sum(), rtol=1e-13, atol=0)
    # tempering: spread 60 > scale 10 -> beta = 10 / (max - mean)
    lnw = rng.normal(0, 20.0, n)
    beta = 10.0 / (lnw.max() - lnw.mean())
    P_ra, _ = orc.hist_refit(bins, lnw, nb, floor=0.25, scale=10.0)
    w = np.exp(beta * (lnw - lnw.max()))
    want = 0.75 * np.bincount(bins[0], w, nb) / w.sum() + 0.25 / nb
    assert np.allclose(P_ra, want, rtol=1e-12)
    assert abs(P_ra.sum() - 1) < 1e-13 and P_ra.min() >= 0.25 / nb
