"""The allocation-free integrate (ile_integrate_dev_noalloc) against
ile_integrate_dev, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the six
result fields (ln L_marg, n_eff and the rest of Eq. (4)'s reduction) must
agree bit for bit.  The allocation-free form keeps its workspace in one
fixed array per GPU that holds the previous call's contents, so every test
makes calls in a row with a smaller input after a larger one: leftovers of
the first call must not reach the second.
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


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _inputs(n, seed):
    s, lp = synth.prior_samples(n, seed)
    rng = np.random.default_rng(seed + 1)
    lq = lp + rng.normal(0.0, 0.3, n)   # a proposal other than the prior
    return s, lp, lq


def _both(torch, ctx, s, lp, lq):
    n = s.shape[1]
    S, P, Q = (_dev(torch, x) for x in (s, lp, lq))
    r_na = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
    r_ref = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()   # the copies and fills above run on torch's stream
    ctx.integrate_dev_noalloc(S, P, Q, n, r_na)
    ctx.sync()
    ctx.integrate_dev(S, P, Q, n, r_ref)
    ctx.sync()
    return r_na.cpu().numpy(), r_ref.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_integrate_dev(torch, prec):
    """Three detectors, 21 modes, 1601 bins: the largest input the fixed
    workspace takes, then a ragged small one."""
    inst = synth.config2()
    print(f"noalloc {prec}: 3 det, 21 modes, n_t 1601", flush=True)
    with ile.Context(inst, precision=prec) as ctx:
        for n, seed in ((ile.NOALLOC_MAX_N, 7101), (12_345, 7102)):
            print(f"  N = {n}", flush=True)
            a, b = _both(torch, ctx, *_inputs(n, seed))
            assert np.all(np.isfinite(a)), a
            assert a[5] == n
            assert np.array_equal(a, b), (n, a, b)


def test_noalloc_contexts_share_the_workspace(torch):
    """Two contexts of different shapes (2 detectors and 5 modes; 3 and 9)
    on one GPU, called one after the other: each matches its own
    ile_integrate_dev, the second call of each smaller than the first."""
    i1 = synth.config1()
    i2 = synth.make_instance(["D1", "D2", "D3"], 9, 4096, 4096.0, 401, 7203)
    with ile.Context(i1) as c1, ile.Context(i2) as c2:
        for n, seed in ((60_001, 7301), (40_000, 7302), (513, 7303), (1, 7304)):
            for c in (c1, c2):
                a, b = _both(torch, c, *_inputs(n, seed))
                assert a[5] == n
                assert np.array_equal(a, b), (n, a, b)


def test_noalloc_refuses_more_than_its_limit(torch):
    """N above ILE_NOALLOC_MAX_N is refused before anything runs; N = 0
    gives the same empty result as ile_integrate_dev."""
    inst = synth.config1()
    with ile.Context(inst) as ctx:
        n = ile.NOALLOC_MAX_N + 1
        S = torch.zeros((7, n), dtype=torch.float64, device="cuda")
        r = torch.full((6,), -3.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(ile.IleError, match="allocation-free limit"):
            ctx.integrate_dev_noalloc(S, None, None, n, r)
        ctx.sync()
        assert np.all(r.cpu().numpy() == -3.0)
        e = np.zeros((7, 0))
        a, b = _both(torch, ctx, e, np.zeros(0), np.zeros(0))
        assert np.array_equal(a, b, equal_nan=True)
        assert a[5] == 0


def test_noalloc_under_graph_capture(torch):
    """The allocation-free call recorded into a HIP graph (torch's graph
    capture on the context's own stream) and replayed three times on new
    samples written in place between the replays, with eager calls of the
    library and synchronizations in between: every replay equals
    ile_integrate_dev on the same samples, bit for bit."""
    inst = synth.config1()
    n = 20_000
    st = torch.cuda.Stream()
    with ile.Context(inst, stream=st.cuda_stream) as ctx:
        S, P, Q = (_dev(torch, x) for x in _inputs(n, 7401))
        r_g = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
        r_ref = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        # an eager call first: the kernels' LDS limits are set outside the capture
        ctx.integrate_dev_noalloc(S, P, Q, n, r_g)
        ctx.sync()
        print("capture", flush=True)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st, capture_error_mode="relaxed"):
            ctx.integrate_dev_noalloc(S, P, Q, n, r_g)
        for seed in (7402, 7403, 7404):
            print(f"replay on the samples of seed {seed}", flush=True)
            for dst, src in zip((S, P, Q), _inputs(n, seed)):
                dst.copy_(_dev(torch, src))
            r_g.fill_(np.nan)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = r_g.cpu().numpy()
            ctx.integrate_dev(S, P, Q, n, r_ref)
            ctx.sync()
            want = r_ref.cpu().numpy()
            assert np.all(np.isfinite(got)) and got[5] == n
            assert np.array_equal(got, want), (seed, got, want)
