"""Proposal reuse across intrinsic points: the Monte Carlo integrator carried
from one intrinsic point to the next, as the paper reuses its adaptive
integrator for each lambda (Sec. II.C; Sec. III.C for the gain on BNS).

Learned runs over a sequence of points on one GPU and one stream.  With
warm=True the network and the sky histograms of point p seed point p+1:
ile_hist_get / ile_hist_set move the histograms, and ile_run with warm = 1
draws the training rounds from the carried-over mixture and starts training
from its weights.  With warm=False every point starts cold.  This module only
sequences library calls on the host; every step runs in the library's
kernels."""
import time

from . import combined, ile


def run(points, *, warm=True, seed=61, target=1e4, chunk=100_000, max_samples=20_000_000,
        precision="fp64", eps=0.1, n_bins=50):
    """points: list of parts (synth.lambda_sequence).  Returns one dict per
    point: wall seconds, result fields and the learned-run counters."""
    import torch
    stream = torch.cuda.Stream()
    handle = stream.cuda_stream
    out = []
    prop = None
    hist = None
    try:
        for p, parts in enumerate(points):
            ctx, _ = combined.injected_point(parts, precision, stream=handle)
            with ctx:
                if prop is None or not warm:
                    if prop is not None:
                        prop.close()
                    prop = ile.Proposal(ctx, seed=3)
                reuse = warm and hist is not None
                if reuse:
                    ile.ile_hist_set(ctx.h, *hist)
                t0 = time.perf_counter()
                r = ctx.run(sampler="learned", seed=seed + p, chunk=chunk,
                            max_samples=max_samples, n_eff_target=target, adapt_chunks=3,
                            prop=prop, eps=eps, n_bins=n_bins, reset=not reuse, warm=reuse)
                r["seconds"] = time.perf_counter() - t0
                r["refits"] = r["n_refine_samples"] // chunk
                r["warm"] = reuse
                hist = ile.ile_hist_get(ctx.h, n_bins)
                out.append(r)
    finally:
        if prop is not None:
            prop.close()
    return out
