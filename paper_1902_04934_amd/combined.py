"""The combined form: each intrinsic point gets its own learned proposal; the
draws of all points of a group are evaluated and reduced in one batched
persistent run (ile_batch_run_dev).  A point whose estimate from those draws
has n_eff below n_eff_min falls back: first to up to `retries` further learned
attempts (a proposal trained on a fresh seed, n fresh draws evaluated through
the point's own context), then to the plain adaptive sampler (ile_run,
refitting as it goes) until n_eff_min or its sample budget; it is reported as
failed if it is still below.  Points are processed in groups so that the
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


# seed offset between learned attempts of one point (training and draws)
ATTEMPT_STRIDE = 1 << 32
# training budgets of a point's learned attempts: the first, then one per
# later attempt (the last repeats); a later attempt gets more adaptive rounds,
# larger chunks and more refits, since the points that need one are those
# whose posterior the first attempt did not capture
TRAINING = (dict(adapt_chunks=5, chunk=100_000, refine_rounds=-1),
            dict(adapt_chunks=10, chunk=200_000, refine_rounds=48),
            dict(adapt_chunks=16, chunk=500_000, refine_rounds=48))


def _train(ctx, g, attempt, *, seed, eps, training=TRAINING):
    """Learned attempt `attempt` of point g: adaptive rounds, training,
    refinement and the probe chunk (their draws are in no estimate), with
    budget training[min(attempt, last)].  Returns the Proposal (the caller
    closes it) and the run's result."""
    t = training[min(attempt, len(training) - 1)]
    prop = ile.Proposal(ctx, seed=3 + attempt)
    try:
        r = ctx.run(sampler="learned", seed=seed + g + attempt * ATTEMPT_STRIDE, chunk=t["chunk"],
                    max_samples=t["chunk"], adapt_chunks=t["adapt_chunks"],
                    refine_rounds=t["refine_rounds"], prop=prop, eps=eps)
    except Exception:
        prop.close()
        raise
    return prop, r


def run_group(points, n, *, precision="fp32", seed=51, draw_seed=7001, eps=0.1,
              n_eff_min=1e3, fallback_samples=20_000_000, workers=4, first=0,
              retries=2, training=TRAINING, d_min=synth.D_MIN_MPC, d_max=synth.D_MAX_MPC):
    """One group: train a proposal per point (points: list of
    synth.combined_point parts; global index first + p seeds point p; a
    training run whose probe falls back is repeated on a fresh seed up to
    `retries` times; see TRAINING for the budgets), draw n samples per
    point, evaluate the group in one batched run, then apply the fallback
    chain to the points whose batched estimate has n_eff < n_eff_min.
    Returns (batched results on the draws, per-point info with the final
    estimate, device draws X [P][7][n], ln p, ln q, the Batch, timings)."""
    import torch
    P = len(points)
    X = torch.empty((P, 7, n), dtype=torch.float64, device="cuda")
    lp = torch.empty((P, n), dtype=torch.float64, device="cuda")
    lq = torch.empty((P, n), dtype=torch.float64, device="cuda")
    ctxs, insts, info = [None] * P, [None] * P, [None] * P
    errors = []
    opts = dict(seed=seed, eps=eps, training=training)

    def work(w):
        stream = torch.cuda.Stream()
        try:
            for p in range(w, P, workers):
                g = first + p
                ctx, inst = injected_point(points[p], precision, stream=stream.cuda_stream)
                ctxs[p], insts[p] = ctx, inst
                t0 = time.perf_counter()
                train_ms = 0.0
                for attempt in range(1 + retries):
                    prop, r = _train(ctx, g, attempt, **opts)
                    train_ms += r["train_ms"]
                    if not r["fell_back"] or attempt == retries:
                        break
                    prop.close()
                ds = draw_seed + g + attempt * ATTEMPT_STRIDE
                with prop:
                    if not r["fell_back"]:
                        prop.sample_dev(ds, 0, n, X[p], n, lp[p], lq[p], eps=eps)
                    else:
                        ile.ile_hist_draw_dev(ctx.h, ds, 0, n, d_min, d_max, X[p], n,
                                              lp[p], lq[p])
                    ctx.sync()
                info[p] = dict(point=g, n_lm=len(points[p]["modes"]), n_t=points[p]["n_t"],
                               attempts=attempt + 1, probe_fell_back=int(r["fell_back"]),
                               train_ms=train_ms, train_s=time.perf_counter() - t0, inst=inst)
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
        # fallback chain on the draws that form the estimate
        t0 = time.perf_counter()
        fell = {p for p in range(P) if res[p]["n_eff"] < n_eff_min}
        if fell:
            Xr = torch.empty((7, n), dtype=torch.float64, device="cuda")
            lpr = torch.empty(n, dtype=torch.float64, device="cuda")
            lqr = torch.empty(n, dtype=torch.float64, device="cuda")
            out = torch.empty(6, dtype=torch.float64, device="cuda")
        for p in range(P):
            info[p]["batched"] = _estimate(res[p], "learned")
            info[p].update(fell_back=int(p in fell), retried=0)
            if p not in fell:
                info[p]["final"] = info[p]["batched"]
                continue
            g, ctx = first + p, ctxs[p]
            final = None
            for k in range(retries):
                attempt = info[p]["attempts"] + k
                info[p]["retried"] = k + 1
                prop, r = _train(ctx, g, attempt, **opts)
                with prop:
                    if r["fell_back"]:
                        continue
                    prop.sample_dev(draw_seed + g + attempt * ATTEMPT_STRIDE, 0, n, Xr, n, lpr,
                                    lqr, eps=eps)
                    ctx.integrate_dev(Xr, lpr, lqr, n, out)
                    ctx.sync()
                v = out.cpu().numpy()
                if v[1] >= n_eff_min:
                    final = dict(ln_L_marg=float(v[0]), n_eff=float(v[1]),
                                 sigma_ln_L=float(v[3]), n_samples=int(v[5]),
                                 source="learned-retry")
                    break
            if final is None:
                r = ctx.run(sampler="adaptive", seed=draw_seed + g + (1 << 40),
                            chunk=1_000_000, max_samples=fallback_samples,
                            n_eff_target=n_eff_min, adapt_chunks=-1, d_min=d_min, d_max=d_max)
                final = _estimate(r, "adaptive")
            info[p]["final"] = final
        t_fallback = time.perf_counter() - t0
    finally:
        for c in ctxs:
            if c is not None:
                c.close()
    for i in info:
        i["failed"] = int(i["final"]["n_eff"] < n_eff_min)
    return res, info, X, lp, lq, batch, dict(train_s=t_train, eval_s=t_eval,
                                              eval_graph_ms=graph_ms, fallback_s=t_fallback)


def run(points, n, *, group=256, progress=None, first=0, **kw):
    """All points in groups of `group` (see run_group; points[i] has global
    index first + i); the draws and the batch of a group are released before
    the next.  progress: a file to which a line is written after each group,
    or None.  Returns (per-point info with its final estimate, without the
    host instance; per-group timings)."""
    out, times = [], []
    for g0 in range(0, len(points), group):
        res, info, X, lp, lq, batch, t = run_group(points[g0:g0 + group], n, first=first + g0,
                                                   **kw)
        batch.close()
        del X, lp, lq
        for i in info:
            i.pop("inst", None)
        out.extend(info)
        times.append(t)
        if progress is not None:
            print(f"combined: points {first + g0}..{first + g0 + len(info) - 1} done, "
                  f"fell back {sum(i['fell_back'] for i in info)}, "
                  f"retried {sum(i['retried'] for i in info)}, "
                  f"failed {sum(i['failed'] for i in info)}, {t}", file=progress, flush=True)
    return out, times
