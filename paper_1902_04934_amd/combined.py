"""The combined form: each intrinsic point gets its own learned proposal; the
draws of all points of a group are evaluated and reduced in one batched
persistent run (ile_batch_run_dev); a point whose estimate from those draws
has n_eff below n_eff_min falls back to the plain adaptive sampler (ile_run,
refitting as it goes) until n_eff_min or its sample budget, and is reported
as failed if it is still below.  Points are processed in groups so that the
draws of a group fit the device (a group of G points holds G x n x 9
doubles); the proposals of a group are trained concurrently on `workers`
streams.  This module only sequences library calls on the host; every step
runs in the library's kernels."""
import threading
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


def _estimate(r, source):
    return dict(ln_L_marg=r["ln_L_marg"], n_eff=r["n_eff"], sigma_ln_L=r["sigma_ln_L"],
                n_samples=r["n_samples"], source=source)


def run_group(points, n, *, precision="fp32", seed=51, draw_seed=7001, eps=0.1,
              n_eff_min=1e3, fallback_samples=20_000_000, workers=4, first=0,
              d_min=synth.D_MIN_MPC, d_max=synth.D_MAX_MPC):
    """One group: train a proposal per point (points: list of
    synth.combined_point parts; global index first + p seeds point p), draw
    n samples per point, evaluate the group in one batched run, then apply
    the fallback to the points whose batched estimate has n_eff < n_eff_min.
    Returns (batched results on the draws, per-point info with the final
    estimate, device draws X [P][7][n], ln p, ln q, the Batch, timings)."""
    import torch
    P = len(points)
    X = torch.empty((P, 7, n), dtype=torch.float64, device="cuda")
    lp = torch.empty((P, n), dtype=torch.float64, device="cuda")
    lq = torch.empty((P, n), dtype=torch.float64, device="cuda")
    ctxs, insts, info = [None] * P, [None] * P, [None] * P
    errors = []

    def work(w):
        stream = torch.cuda.Stream()
        try:
            for p in range(w, P, workers):
                g = first + p
                ctx, inst = injected_point(points[p], precision, stream=stream.cuda_stream)
                ctxs[p], insts[p] = ctx, inst
                t0 = time.perf_counter()
                with ile.Proposal(ctx, seed=3) as prop:
                    # adaptive rounds, training, refinement and the probe chunk
                    # (their draws are not part of any estimate)
                    r = ctx.run(sampler="learned", seed=seed + g, chunk=100_000,
                                max_samples=100_000, adapt_chunks=3, prop=prop, eps=eps)
                    if not r["fell_back"]:
                        prop.sample_dev(draw_seed + g, 0, n, X[p], n, lp[p], lq[p], eps=eps)
                    else:
                        ile.ile_hist_draw_dev(ctx.h, draw_seed + g, 0, n, d_min, d_max, X[p], n,
                                              lp[p], lq[p])
                    ctx.sync()
                info[p] = dict(point=g, n_lm=len(points[p]["modes"]), n_t=points[p]["n_t"],
                               probe_fell_back=int(r["fell_back"]), train_ms=r["train_ms"],
                               train_s=time.perf_counter() - t0, inst=inst)
        except Exception as e:   # re-raised on the calling thread
            errors.append(e)

    t0 = time.perf_counter()
    threads = [threading.Thread(target=work, args=(w,)) for w in range(min(workers, P))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    try:
        if errors:
            raise errors[0]
        t_train = time.perf_counter() - t0
        batch = ile.Batch(precision)
        for inst in insts:
            batch.add_point(inst)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = batch.run_dev(n, X, lp, lq)
        t_eval = time.perf_counter() - t0
        graph_ms = batch.last_ms()
        # fallback on the draws that form the estimate
        t0 = time.perf_counter()
        for p in range(P):
            info[p]["batched"] = _estimate(res[p], "learned")
            if res[p]["n_eff"] >= n_eff_min:
                info[p].update(fell_back=0, final=info[p]["batched"])
                continue
            r = ctxs[p].run(sampler="adaptive", seed=draw_seed + first + p + (1 << 40),
                            chunk=1_000_000, max_samples=fallback_samples,
                            n_eff_target=n_eff_min, adapt_chunks=-1, d_min=d_min, d_max=d_max)
            info[p].update(fell_back=1, final=_estimate(r, "adaptive"))
        t_fallback = time.perf_counter() - t0
    finally:
        for c in ctxs:
            if c is not None:
                c.close()
    for i in info:
        i["failed"] = int(i["final"]["n_eff"] < n_eff_min)
    return res, info, X, lp, lq, batch, dict(train_s=t_train, eval_s=t_eval,
                                              eval_graph_ms=graph_ms, fallback_s=t_fallback)


def run(points, n, *, group=256, progress=None, **kw):
    """All points in groups of `group` (see run_group); the draws and the
    batch of a group are released before the next.  progress: a file to
    which a line is written after each group, or None.  Returns (per-point
    info with its final estimate, without the host instance; per-group
    timings)."""
    out, times = [], []
    for g0 in range(0, len(points), group):
        res, info, X, lp, lq, batch, t = run_group(points[g0:g0 + group], n, first=g0, **kw)
        batch.close()
        del X, lp, lq
        for i in info:
            i.pop("inst", None)
        out.extend(info)
        times.append(t)
        if progress is not None:
            print(f"combined: points {g0}..{g0 + len(info) - 1} done, "
                  f"fell back {sum(i['fell_back'] for i in info)}, "
                  f"failed {sum(i['failed'] for i in info)}, {t}", file=progress, flush=True)
    return out, times
