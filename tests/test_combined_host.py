"""Host logic of the combined form's fallback chain (no GPU): the library
calls are replaced by scripted stand-ins, so that each point's learned
attempts have a chosen probe outcome and a chosen n_eff on their draws.
Checks which draws form each estimate and which source the final estimate
comes from: the batched learned draws, a learned retry on a fresh seed, or
the plain adaptive sampler."""
import sys
import types

import numpy as np
import pytest

from paper_1902_04934_amd import combined

SEED, DRAW_SEED = 51, 7001


class T:
    """A stand-in device tensor (a numpy array)."""

    def __init__(self, a):
        self.a = a

    def __getitem__(self, k):
        return T(self.a[k])

    def cpu(self):
        return self

    def numpy(self):
        return self.a


def fake_torch():
    m = types.ModuleType("torch")
    m.float64 = np.float64
    m.empty = lambda shape, dtype=None, device=None: T(np.zeros(shape))
    m.cuda = types.SimpleNamespace(Stream=lambda: types.SimpleNamespace(cuda_stream=None),
                                   synchronize=lambda: None)
    return m


class Script:
    """attempts[g]: per learned attempt of point g, (probe fell back, n_eff
    of that proposal's draws); adaptive[g]: the plain sampler's n_eff."""

    def __init__(self, attempts, adaptive):
        self.attempts, self.adaptive = attempts, adaptive
        self.calls = []

    def attempt_of(self, g, seed, base):
        k, r = divmod(seed - base - g, combined.ATTEMPT_STRIDE)
        assert r == 0
        return k


class Ctx:
    def __init__(self, script, g):
        self.s, self.g, self.h = script, g, object()

    def run(self, sampler, seed, **kw):
        self.s.calls.append((self.g, sampler))
        if sampler == "learned":
            k = self.s.attempt_of(self.g, seed, SEED)
            # attempt k trains on the k-th budget (the last one repeats)
            t = combined.TRAINING[min(k, len(combined.TRAINING) - 1)]
            assert (kw["chunk"], kw["adapt_chunks"], kw["refine_rounds"]) == \
                (t["chunk"], t["adapt_chunks"], t["refine_rounds"])
            kw["prop"].attempt = k
            return dict(fell_back=int(self.s.attempts[self.g][k][0]), train_ms=1.0)
        assert sampler == "adaptive" and kw["n_eff_target"] == 1e3
        return dict(ln_L_marg=-2.0, n_eff=self.s.adaptive[self.g], sigma_ln_L=0.5,
                    n_samples=kw["max_samples"])

    def integrate_dev(self, X, lp, lq, n, out):
        k = int(X.a[0, 0])
        out.a[:] = [-1.0, self.s.attempts[self.g][k][1], 0.0, 0.01, 0.0, n]

    def sync(self):
        pass

    def close(self):
        pass


class Prop:
    def __init__(self, ctx, seed):
        self.ctx, self.attempt = ctx, None

    def sample_dev(self, seed, first, n, x, ld, lp, lq, eps=0.0):
        g = self.ctx.g
        assert seed == DRAW_SEED + g + self.attempt * combined.ATTEMPT_STRIDE
        x.a[...] = self.attempt

    def close(self):
        pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    def __init__(self, script):
        self.s, self.g = script, []

    def add_point(self, inst):
        self.g.append(inst)

    def run_dev(self, n, X, lp, lq):
        out = []
        for p, g in enumerate(self.g):
            k = int(X.a[p, 0, 0])
            neff = 3.0 if k < 0 else self.s.attempts[g][k][1]
            out.append(dict(ln_L_marg=0.0, n_eff=neff, sigma_ln_L=0.01, n_samples=n))
        return out

    def last_ms(self):
        return 1.0

    def close(self):
        pass


@pytest.fixture
def chain(monkeypatch):
    def setup(attempts, adaptive):
        s = Script(attempts, adaptive)
        monkeypatch.setitem(sys.modules, "torch", fake_torch())
        monkeypatch.setattr(combined, "injected_point",
                            lambda parts, precision, stream=None: (Ctx(s, parts["g"]), parts["g"]))

        def hist_draw(h, seed, first, n, d0, d1, x, ld, lp, lq):
            x.a[...] = -1
        fake_ile = types.SimpleNamespace(Proposal=Prop, ile_hist_draw_dev=hist_draw,
                                         Batch=lambda precision: Batch(s))
        monkeypatch.setattr(combined, "ile", fake_ile)
        pts = [dict(g=g, modes=[(2, 2)], n_t=3) for g in range(len(attempts))]
        res, info, *_ = combined.run_group(pts, 4, seed=SEED, draw_seed=DRAW_SEED, workers=2,
                                           retries=2)
        return s, res, info
    return setup


def test_fallback_chain_sources(chain):
    attempts = [
        [(0, 5e3)],                        # passes on its first draws
        [(1, 0), (0, 2e3)],                # probe falls back once; retrained
        [(0, 10.0), (0, 4e3)],             # draws fail; first retry passes
        [(0, 10.0), (1, 0), (0, 20.0)],    # draws fail; both retries fail
        [(1, 0), (1, 0), (1, 0), (0, 1), (0, 1)],  # every probe falls back
    ]
    s, res, info = chain(attempts, adaptive={3: 1.5e3, 4: 7.0})
    src = [i["final"]["source"] for i in info]
    assert src == ["learned", "learned", "learned-retry", "adaptive", "adaptive"]
    assert [i["attempts"] for i in info] == [1, 2, 1, 1, 3]
    assert [i["probe_fell_back"] for i in info] == [0, 0, 0, 0, 1]
    assert [i["fell_back"] for i in info] == [0, 0, 1, 1, 1]
    assert [i["retried"] for i in info] == [0, 0, 1, 2, 2]
    assert [i["failed"] for i in info] == [0, 0, 0, 0, 1]
    # the batched estimate is the first attempt whose probe passed
    assert [r["n_eff"] for r in res] == [5e3, 2e3, 10.0, 10.0, 3.0]
    assert info[2]["final"]["n_eff"] == 4e3 and info[2]["final"]["n_samples"] == 4
    assert info[1]["final"] is info[1]["batched"]
    # the plain sampler runs only after the learned retries
    adaptive = [g for g, smp in s.calls if smp == "adaptive"]
    assert adaptive == [3, 4]


def test_no_retries_goes_straight_to_adaptive(chain, monkeypatch):
    s = Script([[(0, 10.0), (0, 5e3)]], adaptive={0: 2e3})
    monkeypatch.setitem(sys.modules, "torch", fake_torch())
    monkeypatch.setattr(combined, "injected_point",
                        lambda parts, precision, stream=None: (Ctx(s, 0), 0))
    monkeypatch.setattr(combined, "ile", types.SimpleNamespace(
        Proposal=Prop, ile_hist_draw_dev=None, Batch=lambda precision: Batch(s)))
    res, info, *_ = combined.run_group([dict(g=0, modes=[(2, 2)], n_t=3)], 4, seed=SEED,
                                       draw_seed=DRAW_SEED, retries=0)
    assert info[0]["final"]["source"] == "adaptive" and info[0]["retried"] == 0
    assert info[0]["failed"] == 0
