"""The combined form: each intrinsic point gets its own learned proposal
(ile_run with sampler LEARNED, plain adaptive fallback when its first
estimation chunk has n_eff < 1e3), each point's draws go to one device
buffer [P][7][n] (ile_prop_sample_dev, or ile_hist_draw_dev for a point
that fell back), and one batched persistent run evaluates and reduces all
points together (ile_batch_run_dev).  This module only sequences library
calls on the host; every step runs in the library's kernels."""
import time

import numpy as np

from . import ile, synth


def injected_point(parts, precision="fp32", stream=None):
    """A context holding the device injection of one point (its Q, U, V built
    on the device) and the host Instance with the same Q, U, V.  stream: a
    hipStream_t handle for the context (None: its own)."""
    n_lm, n_q, nd = len(parts["modes"]), parts["n_q"], len(parts["dets"])
    base = synth.Instance(dets=parts["dets"], modes=parts["modes"], srate_hz=parts["srate_hz"],
                          n_t=parts["n_t"], Q=np.zeros((nd, n_lm, n_q), complex),
                          U=np.zeros((nd, n_lm, n_lm), complex),
                          V=np.zeros((nd, n_lm, n_lm), complex))
    ctx = ile.Context(base, precision=precision, stream=stream)
    rho2, dinj, Q, U, V = ile.ile_inject(ctx.h, parts["h_lm"], base.t0_s, base.dets,
                                         parts["theta_inj"], parts["snr"], want_data=True)
    inst = synth.Instance(dets=base.dets, modes=base.modes, srate_hz=base.srate_hz,
                          n_t=base.n_t, Q=Q, U=U, V=V,
                          meta=dict(rho2=rho2, d_inj=dinj))
    return ctx, inst


def run(points, n, *, precision="fp32", seed=51, draw_seed=7001, eps=0.1,
        d_min=synth.D_MIN_MPC, d_max=synth.D_MAX_MPC):
    """Train a proposal per point (points: list of combined_point parts), draw
    n samples per point and evaluate all points in one batched run.
    Returns (per-point results, per-point info, device draws X [P][7][n],
    ln p, ln q, the Batch, timings)."""
    import torch
    P = len(points)
    X = torch.empty((P, 7, n), dtype=torch.float64, device="cuda")
    lp = torch.empty((P, n), dtype=torch.float64, device="cuda")
    lq = torch.empty((P, n), dtype=torch.float64, device="cuda")
    batch = ile.Batch(precision)
    info = []
    t_train = time.perf_counter()
    for p, parts in enumerate(points):
        ctx, inst = injected_point(parts, precision)
        batch.add_point(inst)
        with ctx, ile.Proposal(ctx, seed=3) as prop:
            t0 = time.perf_counter()
            # adaptive rounds, training, refinement and one estimation chunk,
            # whose n_eff decides the fallback; its estimate is not used
            r = ctx.run(sampler="learned", seed=seed + p, chunk=100_000, max_samples=100_000,
                        adapt_chunks=3, prop=prop, eps=eps)
            if not r["fell_back"]:
                prop.sample_dev(draw_seed + p, 0, n, X[p], n, lp[p], lq[p], eps=eps)
            else:
                ile.ile_hist_draw_dev(ctx.h, draw_seed + p, 0, n, d_min, d_max, X[p], n,
                                      lp[p], lq[p])
            ctx.sync()
            info.append(dict(point=p, n_lm=len(parts["modes"]), n_t=parts["n_t"],
                             fell_back=int(r["fell_back"]), seconds=time.perf_counter() - t0,
                             train_ms=r["train_ms"], inst=inst))
    t_train = time.perf_counter() - t_train
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.run_dev(n, X, lp, lq)
    t_eval = time.perf_counter() - t0
    return res, info, X, lp, lq, batch, dict(train_s=t_train, eval_s=t_eval,
                                              eval_graph_ms=batch.last_ms())
