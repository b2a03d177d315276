"""Pins of the oracle's extrinsic harvest (Sec. V: joint extrinsic posterior
draws from a final Monte Carlo iteration; Eq. (3) at fixed intrinsic
parameters) against what the definition and the physics fix:

* equal weights: the inverse-CDF pick is floor(u N) (closed form);
* zero-weight samples (ln p = -inf) are never drawn, a lone weight always;
* the two-stage draw (sample by its Eq. (4) weight, then bin given sample)
  has the marginals of the joint table exp(ln p - ln q + L_alpha,j)
  normalized over all (alpha, j) at once (chi-square);
* on a zero-noise injection the harvested times sit at the injected time,
  whatever the sample's t_ref (pins the bin-to-time mapping and its sign).
"""
import numpy as np
import pytest
from scipy import stats

from paper_1902_04934_amd import synth


def _instance(orc, n_t=21, snr=None, seed=31):
    from test_oracle_pins import chirp_modes
    rng = np.random.default_rng(seed)
    base = synth.make_instance(["D1", "D2", "D3"], 9, 1024, 1024.0, n_t, seed)
    h = chirp_modes(base.n_lm, base.n_q, rng, base.srate_hz)
    th_inj = np.array([1.1, 0.3, 0.7, 2.0, 0.4, 150.0, 0.0031])
    inst, _, _ = orc.injection_instance(base, h, th_inj, snr=snr)
    return inst, th_inj


def _near(th_inj, n, rng, t_spread):
    s = np.repeat(th_inj[:, None], n, axis=1).copy()
    s[:5] += rng.normal(0, 0.03, (5, n))
    s[4] = np.clip(s[4], -1, 1)
    s[5] *= np.exp(rng.normal(0, 0.05, n))
    s[6] += rng.uniform(-t_spread, t_spread, n)
    return s


def test_inverse_cdf_equal_weights_is_floor(orc):
    n = 37
    c = np.cumsum(np.ones(n))
    for u in np.linspace(0, 1, 1001, endpoint=False):
        assert orc.inverse_cdf(c, u * c[-1]) == int(np.floor(u * n))


def test_inverse_cdf_top_and_zero_tail(orc):
    c = np.cumsum([0.0, 2.0, 1.0, 0.0, 0.0])
    assert orc.inverse_cdf(c, 0.0) == 1          # first weight is zero
    assert orc.inverse_cdf(c, c[-1]) == 2        # rounding to the total
    assert orc.inverse_cdf(c, 1.999999) == 1
    assert orc.inverse_cdf(c, 2.0) == 2


def test_zero_weight_never_drawn_single_weight_always(orc):
    inst, th = _instance(orc)
    ctx = orc.Ctx(inst)
    rng = np.random.default_rng(3)
    s = _near(th, 8, rng, 2e-3)
    lp = np.full(8, -np.inf)
    lp[5] = 0.0
    u = rng.uniform(size=(2, 50))
    idx, _, theta = orc.harvest(ctx, s, lp, np.zeros(8), u)
    assert np.all(idx == 5)
    assert np.array_equal(theta[:6], np.repeat(s[:6, 5:6], 50, axis=1))


def test_two_stage_draw_matches_joint_table(orc):
    """The harvest's marginals over samples and over bins equal those of the
    joint table normalized in one step over all (alpha, j)."""
    inst, th = _instance(orc, n_t=21, snr=4.0)
    ctx = orc.Ctx(inst)
    rng = np.random.default_rng(17)
    n = 12
    s = _near(th, n, rng, 4e-3)
    lp = rng.normal(0, 1.0, n)
    lq = rng.normal(0, 1.0, n)
    table = np.array([ctx.lnL_series(s[:, a]) for a in range(n)]) + (lp - lq)[:, None]
    P = np.exp(table - table.max())
    P /= P.sum()
    n_out = 40000
    u = rng.uniform(size=(2, n_out))
    idx, bins, _ = orc.harvest(ctx, s, lp, lq, u)
    for got, p in ((np.bincount(idx, minlength=n), P.sum(axis=1)),
                   (np.bincount(bins, minlength=inst.n_t), P.sum(axis=0))):
        keep = p * n_out > 5
        exp = p[keep] * n_out
        obs = got[keep].astype(float)
        # pool the sparse cells so the statistic keeps its distribution
        obs = np.append(obs, got[~keep].sum())
        exp = np.append(exp, n_out - exp.sum())
        if exp[-1] < 5:
            obs[-2] += obs[-1]
            exp[-2] += exp[-1]
            obs, exp = obs[:-1], exp[:-1]
        chi2 = float(((obs - exp) ** 2 / exp).sum())
        assert stats.chi2.sf(chi2, obs.size - 1) > 1e-4, chi2
    # the same check fails when the proposal density is left out
    P2 = np.exp(table + lq[:, None] - (table + lq[:, None]).max())
    P2 /= P2.sum()
    cnt = np.bincount(idx, minlength=n)
    chi2_wrong = float(((cnt - P2.sum(axis=1) * n_out) ** 2 / (P2.sum(axis=1) * n_out)).sum())
    assert stats.chi2.sf(chi2_wrong, n - 1) < 1e-6


def test_harvested_time_is_injected_time(orc):
    """Loud zero-noise injection: whatever t_ref a sample carries (within the
    window), the harvested geocentre time is the injected one to within one
    sample."""
    inst, th = _instance(orc, n_t=41, snr=60.0)
    ctx = orc.Ctx(inst)
    rng = np.random.default_rng(5)
    n = 16
    s = np.repeat(th[:, None], n, axis=1).copy()
    s[6] += rng.integers(-12, 13, n) / inst.srate_hz
    u = rng.uniform(size=(2, 400))
    idx, bins, theta = orc.harvest(ctx, s, np.zeros(n), np.zeros(n), u)
    dt = 1.0 / inst.srate_hz
    assert np.all(np.abs(theta[6] - th[6]) <= dt * (1 + 1e-9))
    assert np.mean(np.abs(theta[6] - th[6]) < 0.5 * dt) > 0.9
    # bin j and t_ref are tied by t = t_ref + (j - h) dt
    h = (inst.n_t - 1) // 2
    assert np.allclose(theta[6], s[6, idx] + (bins - h) * dt, rtol=0, atol=1e-15)


def test_invalid_inputs_raise(orc):
    inst, th = _instance(orc)
    ctx = orc.Ctx(inst)
    s = _near(th, 4, np.random.default_rng(1), 1e-3)
    with pytest.raises(ValueError):
        orc.harvest(ctx, s, np.full(4, -np.inf), np.zeros(4), np.zeros((2, 3)))
