#!/usr/bin/env python3
"""Benchmark of the ILE likelihood hot path on one MI355X.

One step = the whole hot path over one batch: draw the batch of extrinsic
samples from the prior on the device (Philox), evaluate ln L_margT for every
sample (window starts, ordering, fused contraction + FP64 time
log-sum-exp), and reduce to ln L_marg and n_eff; only the 6-number result
crosses to the host.  Q, U, V are resident in HBM before timing starts.

Workload (default): 3 detectors, 21 modes (l = 2..4), Q of 16384 complex
points at 16384 Hz, 1e6 prior samples, 1601 time bins, FP64 -- the plain
at-scale single-point configuration.  Synthetic data (seeded stand-ins).

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lnL evals/s (sample×time-bin) + N_eff/s learned vs plain at 1e-3, 1 GPU"
FP64_PEAK_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 lanes x 2 flop (FMA)
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0  # dense matrix peak


KERNEL_SOURCES = ("paper_1902_04934_amd/csrc/ile_kernels.hip",
                  "paper_1902_04934_amd/csrc/ile_internal.h")


def kernel_source_hash():
    """sha256 of the contraction kernel's sources (identifies the kernel the
    committed counter readings belong to)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(precision, engine, threads):
    """HBM bytes of one contraction launch (the terms pass and the tiles for
    the phased engine) from the committed rocprofv3 summary of this workload
    (FETCH_SIZE + WRITE_SIZE, calibrated), if it was taken on the current
    kernel sources, engine and launch shape; else None."""
    import glob
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        fields = {}
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic-record: "):
                    for kv in line[len("traffic-record: "):].split():
                        k, _, v = kv.partition("=")
                        fields[k] = v
        if (fields.get("source_sha256") == want and fields.get("precision") == precision
                and fields.get("engine") == engine and fields.get("threads") == str(threads)
                and "bytes" in fields):
            return int(fields["bytes"])
    return None


def flops_per_sample(n_det, n_lm, n_t):
    """Algorithmic flops of one sample: the window contraction (Re(conj(c) Q)
    = 2 FMA = 4 flop per detector, mode and bin) plus the quadratic term
    (16 flop per detector and mode pair)."""
    return 4 * n_det * n_lm * n_t + 16 * n_det * n_lm * n_lm


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(octx, n_total, n_t, seed, threads, target_s):
    """sample*bin/s of the FP64 oracle on the first M prior draws of the
    stream, M sized for about target_s seconds from a first timing of 2000."""
    from oracle import oracle as O
    m0 = min(2000, n_total)
    s0, _ = O.prior_draw(seed, 0, m0)
    t = time.perf_counter()
    octx.eval(s0, n_threads=threads)
    dt0 = time.perf_counter() - t
    m = int(min(n_total, max(m0, m0 * target_s / max(dt0, 1e-6))))
    sub, _ = O.prior_draw(seed, 0, m)   # the same draws as the device stream
    t = time.perf_counter()
    octx.eval(sub, n_threads=threads)
    dt = time.perf_counter() - t
    return m * n_t / dt, m, dt


def cpu_baseline(inst, n_total, seed, target_s=8.0):
    """The FP64 oracle on the host cores: the benchmark workload with all
    threads (the reported value) and with one, and the small two-detector
    workload (2 detectors, 5 modes, 4096 Hz, 201 bins, 1e4 samples) with both,
    each on a bounded sample of the same prior stream (about target_s seconds
    of CPU work per timing)."""
    from oracle import oracle as O
    from paper_1902_04934_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    rate, m, dt = _oracle_rate(O.Ctx(inst), n_total, inst.n_t, seed, threads, target_s)
    rate1, m1, dt1 = _oracle_rate(O.Ctx(inst), n_total, inst.n_t, seed, 1, target_s)
    i1 = synth.config1()
    n1, seed1 = synth.CONFIG_SAMPLES[1]
    c1 = O.Ctx(i1)
    r1a, m1a, _ = _oracle_rate(c1, n1, i1.n_t, seed1, threads, target_s / 4)
    r1b, m1b, _ = _oracle_rate(c1, n1, i1.n_t, seed1, 1, target_s / 4)
    return {"value": rate, "unit": "sample*bin/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} of the {n_total} prior samples, all {inst.n_t} bins, "
                      f"FP64 C oracle with OpenMP ({dt:.1f} s)",
            "cpu_model": cpu_model(),
            "one_thread": {"value": rate1, "sample": f"first {m1} samples ({dt1:.1f} s)"},
            "small_workload": {"workload": "2 detectors, 5 modes (l=2), Q 4096 points at "
                                           "4096 Hz, 201 time bins",
                               "all_threads": r1a, "one_thread": r1b,
                               "samples": [m1a, m1b]}}


LEARNED_SEEDS = tuple(range(41, 49))


def learned_leg(target=1e4):
    """The learned proposal against the plain adaptive sampler on the zero-noise
    injection workload (3 detectors, 9 modes, 16384 points at 16384 Hz, 1601
    bins, network SNR 20): wall time of each to n_eff = target, n_eff/s, and
    their ln L_marg.  The learned sampler (run defaults) is timed on eight
    run seeds: each seed trains its own network on its own draws, so the
    spread over seeds is the spread a user sees; the headline is the median.
    Every estimate is compared with an independent reference (a learned run
    on seed 9001 continued to 3e8 draws of its defensive mixture, sigma about
    3e-5): the difference and the combined standard error per run."""
    import numpy as np
    from paper_1902_04934_amd import ile, synth
    c = synth.config4_parts()
    base = synth.Instance(dets=c["dets"], modes=c["modes"], srate_hz=c["srate_hz"],
                          n_t=c["n_t"], Q=np.zeros((3, 9, c["n_q"]), complex),
                          U=np.zeros((3, 9, 9), complex), V=np.zeros((3, 9, 9), complex))
    out = {"workload": "zero-noise injection at network SNR 20: 3 detectors, 9 modes "
                       "(l=2,3), Q 16384 complex points at 16384 Hz, 1601 time bins, FP64",
           "n_eff_target": target}
    def entry(r, dt):
        return {"seconds": dt, "n_eff": r["n_eff"], "n_eff_per_s": r["n_eff"] / dt,
                "ln_L_marg": r["ln_L_marg"], "sigma_ln_L": r["sigma_ln_L"],
                "samples": r["n_samples"]}

    with ile.Context(base) as ctx:
        rho2, dinj = ile.ile_inject(ctx.h, c["h_lm"], base.t0_s, base.dets, c["theta_inj"],
                                    c["snr"])
        ctx.run(sampler="prior", seed=1, chunk=100_000, max_samples=100_000)   # warm-up
        t0 = time.perf_counter()
        r = ctx.run(sampler="adaptive", adapt_chunks=-1, max_samples=50_000_000, seed=41,
                    chunk=100_000, n_eff_target=target)
        out["plain"] = entry(r, time.perf_counter() - t0)
        runs = []
        for seed in LEARNED_SEEDS:
            with ile.Proposal(ctx, seed=3) as prop:
                t0 = time.perf_counter()
                r = ctx.run(sampler="learned", adapt_chunks=3, max_samples=20_000_000, eps=0.1,
                            seed=seed, chunk=100_000, n_eff_target=target, prop=prop)
                e = entry(r, time.perf_counter() - t0)
            e.update(seed=seed, train_samples=r["n_train_samples"], train_ms=r["train_ms"],
                     fell_back=r["fell_back"])
            runs.append(e)
        # independent reference: a learned run on its own seed, then 3e8 draws
        # of its defensive mixture (unbiased for any covering q)
        with ile.Proposal(ctx, seed=7) as prop:
            t0 = time.perf_counter()
            r = ctx.run(sampler="learned", seed=9001, chunk=1_000_000, max_samples=300_000_000,
                        n_eff_target=1e12, adapt_chunks=3, prop=prop, eps=0.1)
            ref = entry(r, time.perf_counter() - t0)
        out["reference"] = ref
    import statistics
    ok = [e for e in runs if not e["fell_back"] and e["n_eff"] >= target]
    med = statistics.median(e["n_eff_per_s"] for e in runs)
    out["learned"] = {"seeds": list(LEARNED_SEEDS), "reached_target": len(ok),
                      "fell_back": sum(e["fell_back"] for e in runs),
                      "median_n_eff_per_s": med, "runs": runs}
    out["gain_n_eff_per_s_median"] = med / max(out["plain"]["n_eff_per_s"], 1e-30)
    if ok:
        lnls = [e["ln_L_marg"] for e in ok]
        out["ln_L_marg_learned_median"] = statistics.median(lnls)
        out["ln_L_marg_learned_spread"] = max(lnls) - min(lnls)
        out["d_ln_L_marg_vs_plain"] = statistics.median(lnls) - out["plain"]["ln_L_marg"]
    import math
    for e in runs + [out["plain"]]:
        e["d_ln_L_vs_reference"] = e["ln_L_marg"] - ref["ln_L_marg"]
        e["sigma_combined"] = math.hypot(e["sigma_ln_L"], ref["sigma_ln_L"])
    out["within_1e-3_plus_3sigma"] = sum(
        abs(e["d_ln_L_vs_reference"]) <= 1e-3 + 3 * e["sigma_combined"] for e in runs)
    return out


def batched_leg(n_points=256, n=200_000, steps=3, seed=11):
    """The batched form on its workload: 256 intrinsic points with 5, 9, 13 or
    21 modes and 201-1601 bins (by seed), 3 detectors, Q 16384 points in
    FP32, 2e5 prior samples per point, one graph-captured persistent run
    (draw, order, sort, contraction, per-point reduction) at the default
    tuning.  Reports the graph's device time (HIP events) and wall time per
    run, and the throughput in sample x bin per second."""
    from paper_1902_04934_amd import ile, synth
    t0 = time.perf_counter()
    pts = [synth.batched_point(p) for p in range(n_points)]
    t_gen = time.perf_counter() - t0
    work = n * sum(p.n_t for p in pts)
    with ile.Batch("fp32") as b:
        for inst in pts:
            b.add_point(inst)
        b.run(seed, n)
        t0 = time.perf_counter()
        gms = []
        for _ in range(steps):
            res = b.run(seed, n)
            gms.append(b.last_ms())
        wall = 1e3 * (time.perf_counter() - t0) / steps
        tune = b.get_tuning()
    g = sum(gms) / len(gms)
    flops = n * sum(4 * p.n_det * p.n_lm * p.n_t + 16 * p.n_det * p.n_lm ** 2 for p in pts)
    return {"workload": f"{n_points} points (3 detectors, 5-21 modes, 201-1601 bins, Q 16384 "
                        f"points FP32), {n} prior samples each, one graph",
            "graph_ms": g, "wall_ms_per_run": wall, "sample_bins_per_s": work / (g * 1e-3),
            "samples_per_s": n * n_points / (g * 1e-3), "tuning": tune,
            "fp32_tflops": flops / (g * 1e-3) / 1e12,
            "input_generation_s": t_gen,
            "n_eff_min": min(r["n_eff"] for r in res)}


def rom_leg(n=1_000_000, steps=5):
    """Surrogate (linear-basis) form at the benchmark point's shape: its Q,
    U, V as the overlaps of 21 basis functions, 21 physical modes, a seeded
    cubic-in-lambda coefficient table; n joint samples (prior extrinsic draws
    on the device, lambda uniform on [-1, 1]) evaluated and reduced in one
    Monte Carlo over intrinsic and extrinsic parameters.  Reports the wall
    time per step and the contraction's device time."""
    import numpy as np
    import torch
    from paper_1902_04934_amd import ile, synth
    basis = synth.config2()
    rng = np.random.default_rng(91)
    A = (rng.normal(size=(21, 21, 4)) + 1j * rng.normal(size=(21, 21, 4))) / 21
    with ile.Context(basis) as ctx:
        ile.ile_rom_set(ctx.h, synth.MODE_ORDER[:21], A)
        X = torch.empty((8, n), dtype=torch.float64, device="cuda")
        lp = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(92)
        X[7] = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
        torch.cuda.synchronize()
        ctx.draw_prior_dev(93, 0, n, X, n, lp)
        r = torch.empty(6, dtype=torch.float64, device="cuda")
        ile.ile_rom_integrate_dev(ctx.h, X, lp, lp, n, r)
        ctx.sync()
        t0 = time.perf_counter()
        kms = []
        for _ in range(steps):
            ile.ile_rom_integrate_dev(ctx.h, X, lp, lp, n, r)
            ctx.sync()
            kms.append(ctx.last_kernel_ms())
        ms = 1e3 * (time.perf_counter() - t0) / steps
        res = r.cpu().numpy()
    return {"workload": f"surrogate form: 21 basis functions (Q 16384 points at 16384 Hz, 3 "
                        f"detectors, {basis.n_t} bins), 21 physical modes, 4 powers of lambda, "
                        f"{n} joint (lambda, theta) samples",
            "ms_per_step": ms, "kernel_ms": sum(kms) / len(kms),
            "evals_per_s": n * basis.n_t / (ms * 1e-3),
            "ln_L_marg": float(res[0]), "n_eff": float(res[1])}


def qvu_leg(steps=10):
    """Q, U, V built on the device from frequency-domain series at the
    benchmark point's shape (3 detectors, 21 modes, 16384-point grid at
    16384 Hz, band 20-4000 Hz): wall time of the blocking build, the inverse
    FFT's device time, and the build's compulsory HBM bytes (read h, d, S;
    write Q, U, V) over its wall time against the 8 TB/s peak."""
    import numpy as np
    import torch
    from paper_1902_04934_amd import ile, synth
    c = synth.fd_inputs(["D1", "D2", "D3"], 21, 16384, 16384.0, 611)
    nd, nl, n = 3, 21, c["n_q"]
    H = torch.tensor(np.ascontiguousarray(c["h_f"]).view(np.float64), device="cuda")
    D = torch.tensor(np.ascontiguousarray(c["d_f"]).view(np.float64), device="cuda")
    P = torch.tensor(np.ascontiguousarray(c["psd"]), device="cuda")
    Q = torch.empty((nd, nl, 2 * n), dtype=torch.float64, device="cuda")
    U = torch.empty((nd, nl, 2 * nl), dtype=torch.float64, device="cuda")
    V = torch.empty((nd, nl, 2 * nl), dtype=torch.float64, device="cuda")
    h = ile.ile_create(c["dets"], c["modes"], c["srate_hz"], 1601)
    try:
        torch.cuda.synchronize()
        ile.ile_qvu_fd_dev(h, H, D, P, n, c["df"], 20.0, 4000.0, -0.5, Q, U, V)
        t0 = time.perf_counter()
        ffts = []
        for _ in range(steps):
            ile.ile_qvu_fd_dev(h, H, D, P, n, c["df"], 20.0, 4000.0, -0.5, Q, U, V)
            ffts.append(ile.lib().ile_last_kernel_ms(h))
        ms = 1e3 * (time.perf_counter() - t0) / steps
    finally:
        ile.ile_destroy(h)
    nbytes = 16 * n * (nl + nd) + 8 * n * nd + 16 * n * nd * nl + 2 * 16 * nd * nl * nl
    return {"workload": "Q, U, V of 3 detectors x 21 modes on a 16384-point grid "
                        "(16384 Hz), band 20-4000 Hz, FP64",
            "build_ms": ms, "ifft_ms": sum(ffts) / len(ffts), "compulsory_bytes": nbytes,
            "hbm_frac_of_build": nbytes / (ms * 1e-3) / 8e12}


def reuse_leg(n_points=8, target=1e4):
    """Proposal reuse across intrinsic points on a sequence of neighbouring
    points (the learned-proposal workload with the stand-in chirp's f0 and
    fdot stepped by 1% per point): learned runs to n_eff = target, every
    point cold, then the network and histograms carried from point to point
    (warm).  Reports the wall time per point and the largest cold-warm
    difference of ln L_marg in units of their combined standard error."""
    import numpy as np
    from paper_1902_04934_amd import reuse, synth
    pts = synth.lambda_sequence(n_points)
    cold = reuse.run(pts, warm=False, target=target)
    warm = reuse.run(pts, warm=True, target=target)
    def summary(rs):
        return {"seconds": [r["seconds"] for r in rs], "refits": [r["refits"] for r in rs],
                "fell_back": sum(r["fell_back"] for r in rs),
                "n_eff": [r["n_eff"] for r in rs], "ln_L_marg": [r["ln_L_marg"] for r in rs]}
    z = max(abs(c["ln_L_marg"] - w["ln_L_marg"]) / np.hypot(c["sigma_ln_L"], w["sigma_ln_L"])
            for c, w in zip(cold, warm))
    sc = sum(r["seconds"] for r in cold[1:])
    sw = sum(r["seconds"] for r in warm[1:])
    return {"workload": f"{n_points} neighbouring intrinsic points (3 detectors, 9 modes, 1601 "
                        "bins, FP64, injections at network SNR 20), learned runs to "
                        f"n_eff = {target:g}",
            "cold": summary(cold), "warm": summary(warm),
            "seconds_per_point_after_first": {"cold": sc / (n_points - 1),
                                              "warm": sw / (n_points - 1)},
            "speedup_after_first": sc / sw,
            "max_abs_d_ln_L_over_sigma": float(z)}


def combined_leg(n_points=32, n=1_000_000, m_oracle=2000, group=256, first=0):
    """The combined form at the combined workload's per-point shape (3
    detectors, 5-21 modes, 201-1601 bins, 16384-point Q in FP32, 1e6 draws
    per point) on n_points points: a learned proposal per point (trained on
    4 concurrent streams), the draws of a group of points evaluated in one
    batched persistent run, and the fallback chain (up to two learned retries
    on fresh seeds, then the plain adaptive sampler) for every point whose
    n_eff from those draws is below 1e3.  Reports the batched evaluation's
    throughput (HIP events around its graph), the end-to-end wall time, the
    fallback, retry and failure counts, the source of each final estimate,
    and each point's final ln L_marg, n_eff and sigma.  Up to 32 points: one group, with ln L_marg
    against the FP64 oracle on the first m_oracle draws of every point (the
    device value from a batched run of those draws)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1902_04934_amd import combined, synth
    points = [synth.combined_point(p) for p in range(first, first + n_points)]
    work = sum(n * p["n_t"] for p in points)
    t0 = time.perf_counter()
    errs, t_orc = [], 0.0
    if n_points <= 32:
        res, info, X, lp, lq, batch, t = combined.run_group(points, n, first=first)
        times = [t]
        wall = time.perf_counter() - t0
        Xs, lps, lqs = X[:, :, :m_oracle].contiguous(), lp[:, :m_oracle].contiguous(), \
            lq[:, :m_oracle].contiguous()
        sub = batch.run_dev(m_oracle, Xs, lps, lqs)
        t_orc = time.perf_counter()
        for p, parts in enumerate(points):
            inst = info[p]["inst"]
            blank = synth.Instance(dets=inst.dets, modes=inst.modes, srate_hz=inst.srate_hz,
                                   n_t=inst.n_t, Q=np.zeros_like(inst.Q),
                                   U=np.zeros_like(inst.U), V=np.zeros_like(inst.V))
            want, _, _ = O.injection_instance(blank, parts["h_lm"], parts["theta_inj"],
                                              snr=parts["snr"])
            lnL = O.Ctx(want).eval(Xs[p].cpu().numpy())
            ref = O.integrate(lnL, lps[p].cpu().numpy(), lqs[p].cpu().numpy())
            errs.append(abs(sub[p]["ln_L_marg"] - ref["ln_L_marg"]))
        t_orc = time.perf_counter() - t_orc
        batch.close()
    else:
        info, times = combined.run(points, n, group=group, progress=sys.stderr, first=first)
        wall = time.perf_counter() - t0
    graph_ms = sum(t["eval_graph_ms"] for t in times)
    fin = [i["final"] for i in info]
    return {"workload": f"{n_points} injected points from point {first} (3 detectors, 5-21 "
                        f"modes, 201-1601 bins, Q 16384 points FP32), {n} draws per point "
                        f"from per-point learned "
                        f"proposals, batched evaluation in groups of up to {group} points",
            "points": n_points, "first_point": first, "draws_per_point": n,
            "groups": len(times),
            "eval_graph_ms": graph_ms,
            "eval_sample_bins_per_s": work / (graph_ms * 1e-3),
            "train_and_draw_s": sum(t["train_s"] for t in times),
            "fallback_s": sum(t["fallback_s"] for t in times), "wall_s": wall,
            "points_per_s": n_points / wall,
            "fell_back": sum(i["fell_back"] for i in info),
            "probe_retrained": sum(i["attempts"] > 1 for i in info),
            "retries": sum(i["retried"] for i in info),
            "final_source": {k: sum(f["source"] == k for f in fin)
                             for k in ("learned", "learned-retry", "adaptive")},
            "failed": sum(i["failed"] for i in info),
            "n_eff": [f["n_eff"] for f in fin], "ln_L_marg": [f["ln_L_marg"] for f in fin],
            "sigma_ln_L": [f["sigma_ln_L"] for f in fin],
            "oracle_subset_draws": m_oracle if errs else 0,
            "max_abs_d_ln_L_marg_vs_oracle": max(errs) if errs else None, "oracle_s": t_orc}


def harvest_leg(inst, n, seed, n_out=100_000, steps=3, m_check=50):
    """Extrinsic posterior harvest on the benchmark workload as one final
    iteration: n prior draws (proposal = prior, so the sample weight is the
    likelihood) evaluated and reduced to ln L_marg, and n_out joint (sample,
    time bin) draws.  Reports the blocking call's wall time and
    checks m_check draws' bins against the oracle's per-bin series, and every
    draw's parameters against its sample."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_1902_04934_amd import ile
    with ile.Context(inst) as ctx:
        X = torch.empty((7, n), dtype=torch.float64, device="cuda")
        lp = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.draw_prior_dev(seed, 0, n, X, n, lp)
        g = torch.Generator(device="cuda")
        g.manual_seed(seed + 17)
        u = torch.rand((2, n_out), dtype=torch.float64, device="cuda", generator=g)
        idx = torch.empty(n_out, dtype=torch.int64, device="cuda")
        bins = torch.empty(n_out, dtype=torch.int32, device="cuda")
        th = torch.empty((7, n_out), dtype=torch.float64, device="cuda")
        res = torch.empty(6, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()   # u comes from torch's stream, the draws from the context's
        ctx.sync()
        ctx.harvest_dev(X, lp, lp, n, u, n_out, idx, bins, th, res)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.harvest_dev(X, lp, lp, n, u, n_out, idx, bins, th, res)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        xs, ids, bs, ths, us, r = (t.cpu().numpy() for t in (X, idx, bins, th, u, res))
    h = (inst.n_t - 1) // 2
    octx = O.Ctx(inst)
    rng = np.random.default_rng(seed)
    agree = 0
    for k in rng.choice(n_out, m_check, replace=False):
        L = octx.lnL_series(xs[:, ids[k]])
        c = np.cumsum(np.exp(L - L.max()))
        agree += int(O.inverse_cdf(c, us[1, k] * c[-1]) == bs[k])
    consistent = bool(np.array_equal(ths[:6], xs[:6, ids]) and np.array_equal(
        ths[6], xs[6, ids] + (bs.astype(np.int64) - h) / inst.srate_hz))
    return {"workload": f"{n} prior draws of the benchmark point, {n_out} joint "
                        f"(sample, time bin) draws over {inst.n_t} bins",
            "harvest_ms": ms, "draws_per_s": n_out / (ms * 1e-3),
            "ln_L_marg": float(r[0]), "n_eff": float(r[1]),
            "distinct_samples": int(np.unique(ids).size),
            "oracle_bin_checks": m_check, "oracle_bin_agree": agree,
            "params_consistent": consistent}


def precision_forms(inst, n, seed, steps, m_oracle=2000):
    """The bulk contraction in FP64, FP32 and BF16 hi/lo (time marginalization
    and reduction in FP64 in all three) on the same workload: kernel time,
    evaluation rate and fraction of the precision's peak, and the largest
    per-sample |d lnL| / max(1, |lnL|) against the FP64 oracle on the first
    m_oracle prior draws of the run's stream."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_1902_04934_amd import ile
    peak = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS}
    fl = flops_per_sample(inst.n_det, inst.n_lm, inst.n_t) * n
    out = {}
    x = None
    for prec in ("fp64", "fp32", "bf16"):
        with ile.Context(inst, precision=prec) as ctx:
            ctx.run_prior(seed, n)
            kms = []
            for _ in range(steps):
                ctx.run_prior(seed, n)
                kms.append(ctx.last_kernel_ms())
            kernel_ms = sum(kms) / len(kms)
            xd = torch.empty((7, m_oracle), dtype=torch.float64, device="cuda")
            ctx.draw_prior_dev(seed, 0, m_oracle, xd, m_oracle)
            lnd = torch.empty(m_oracle, dtype=torch.float64, device="cuda")
            ctx.eval_dev(xd, m_oracle, lnd)
            ctx.sync()
            got = lnd.cpu().numpy()
            if x is None:
                x = xd.cpu().numpy()
                want = O.Ctx(inst).eval(x)
        rel = np.abs(got - want) / np.maximum(1.0, np.abs(want))
        out[prec] = {"kernel_ms": kernel_ms, "evals_per_s": n * inst.n_t / (kernel_ms * 1e-3),
                     "frac_of_peak": fl / (kernel_ms * 1e-3) / 1e12 / peak[prec],
                     "max_rel_err_lnL_vs_oracle": float(np.max(rel)),
                     "p99_rel_err_lnL_vs_oracle": float(np.percentile(rel, 99))}
    out["oracle_samples"] = m_oracle
    return out


def mode_scaling_leg(n=200_000, steps=3):
    """Contraction time against the number of modes (Sec. III.B: the cost
    grows with the modes) for every engine and precision: 3 detectors, Q of
    16384 points at 16384 Hz, 1601 bins, n prior samples, n_lm in
    {5, 9, 13, 21} (l = 2, then l = 2..3 with |m| <= 1 for 9, ...; the
    stand-in instances of synth.make_instance).  Per engine: event-timed
    milliseconds per launch scaled to 1e6 samples, and the fraction of the
    precision's peak at the algorithmic flop count."""
    from paper_1902_04934_amd import ile, synth
    peak = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS}
    rows = []
    for n_lm in (5, 9, 13, 21):
        inst = synth.make_instance(["D1", "D2", "D3"], n_lm, 16384, 16384.0, 1601, 3000 + n_lm)
        fl = flops_per_sample(3, n_lm, 1601) * n
        for prec in ("fp64", "fp32"):
            for eng in ("mfma", "pipelined", "valu"):
                with ile.Context(inst, precision=prec, engine=eng) as ctx:
                    ctx.run_prior(5, n)
                    kms = []
                    for _ in range(steps):
                        ctx.run_prior(5, n)
                        kms.append(ctx.last_kernel_ms())
                ms = min(kms)
                rows.append({"n_lm": n_lm, "precision": prec,
                             "engine": "phased" if eng == "mfma" else eng,
                             "ms_per_1e6": ms * 1e6 / n,
                             "frac_of_peak": fl / (ms * 1e-3) / 1e12 / peak[prec]})
    return {"workload": f"3 detectors, Q 16384 points at 16384 Hz, 1601 bins, {n} prior "
                        "samples per launch", "rows": rows}


def latency_leg(calls=50):
    """The small workload as a latency: 2 detectors, 5 modes (l = 2), Q of
    4096 points at 4096 Hz, 201 bins, 1e4 prior samples per call; host wall
    time of one whole call (device prior draw, ordering, contraction,
    reduction, result to the host) and the contraction's event time; then
    the same call as a HIP graph replay (_latency_graph)."""
    import statistics
    from paper_1902_04934_amd import ile, synth
    inst = synth.config1()
    n, seed = synth.CONFIG_SAMPLES[1]
    with ile.Context(inst) as ctx:
        for _ in range(5):
            ctx.run_prior(seed, n)
        walls, kms = [], []
        for _ in range(calls):
            t0 = time.perf_counter()
            r = ctx.run_prior(seed, n)
            walls.append((time.perf_counter() - t0) * 1e3)
            kms.append(ctx.last_kernel_ms())
    walls.sort()
    graph = _latency_graph(inst, n, seed, calls, r)
    return {"workload": "2 detectors, 5 modes (l=2), Q 4096 points at 4096 Hz, "
                        f"{n} prior samples, {inst.n_t} time bins, FP64",
            "calls": calls, "wall_ms_median": statistics.median(walls),
            "wall_ms_p90": walls[int(0.9 * (calls - 1))],
            "kernel_ms_median": statistics.median(kms),
            "ln_L_marg": r["ln_L_marg"], "n_eff": r["n_eff"], "graph": graph}


def _latency_graph(inst, n, seed, calls, eager):
    """The same call recorded once into a HIP graph (the device prior draw,
    then the allocation-free integrate) and replayed per call; wall time of a
    replay plus the result's copy to pinned host memory, and whether the
    replayed result equals the eager call's."""
    import statistics
    import torch
    from paper_1902_04934_amd import ile
    st = torch.cuda.Stream()
    with ile.Context(inst, stream=st.cuda_stream) as ctx:
        X = torch.empty((7, n), dtype=torch.float64, device="cuda")
        r = torch.empty(6, dtype=torch.float64, device="cuda")
        host = torch.empty(6, dtype=torch.float64, pin_memory=True)
        torch.cuda.synchronize()
        ctx.draw_prior_dev(seed, 0, n, X, n)           # eager first: kernel limits set
        ctx.integrate_dev_noalloc(X, None, None, n, r)
        ctx.sync()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st, capture_error_mode="relaxed"):
            ctx.draw_prior_dev(seed, 0, n, X, n)
            ctx.integrate_dev_noalloc(X, None, None, n, r)
        cur = torch.cuda.current_stream()
        walls = []
        for i in range(5 + calls):
            t0 = time.perf_counter()
            g.replay()
            host.copy_(r, non_blocking=True)
            cur.synchronize()
            if i >= 5:
                walls.append((time.perf_counter() - t0) * 1e3)
        res = host.numpy().copy()
    walls.sort()
    return {"wall_ms_median": statistics.median(walls),
            "wall_ms_p90": walls[int(0.9 * (calls - 1))],
            "equals_eager": bool(res[0] == eager["ln_L_marg"] and res[1] == eager["n_eff"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--engine", default=None, choices=["mfma", "pipelined", "valu"],
                    help="contraction engine: mfma = the phased matrix-core engine (the "
                         "default; BF16: the pipelined one), pipelined = producer/consumer "
                         "matrix-core waves, valu = vector FMA")
    ap.add_argument("--threads", type=int, default=None, choices=[128, 192, 256, 512])
    ap.add_argument("--lds-kb", type=int, default=None,
                    help="LDS budget of a phased workgroup in KiB (default by precision)")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the engine x precision x mode-count table")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the small-workload latency leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain sampler comparison")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP64/FP32/BF16 comparison on the same workload")
    ap.add_argument("--no-combined", action="store_true",
                    help="skip the combined-form leg (per-point learned proposals, batched)")
    ap.add_argument("--combined-points", type=int, default=32,
                    help="points of the combined-form leg (4096: the full workload; above "
                         "32 in groups of 256, without the oracle subset check)")
    ap.add_argument("--combined-first", type=int, default=0,
                    help="global index of the combined-form leg's first point (a run of the "
                         "4096-point workload may be split into ranges)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched form on its 256-point workload")
    ap.add_argument("--no-rom", action="store_true",
                    help="skip the surrogate (linear-basis) joint Monte Carlo leg")
    ap.add_argument("--no-qvu", action="store_true",
                    help="skip the frequency-domain Q, U, V construction leg")
    ap.add_argument("--no-reuse", action="store_true",
                    help="skip the proposal-reuse leg (cold vs warm over neighbouring points)")
    ap.add_argument("--no-harvest", action="store_true",
                    help="skip the extrinsic posterior harvest leg")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1902_04934_amd import ile, synth

    inst = synth.config2()
    n_total, seed = synth.CONFIG_SAMPLES[2]
    n = args.samples or n_total
    ctx = ile.Context(inst, precision=args.precision, device=0, engine=args.engine,
                      threads=args.threads, lds_kb=args.lds_kb)
    torch.cuda.synchronize()
    if args.calib_copy:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = a.clone()
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        ctx.run_prior(seed, n)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.run_prior(seed, n)
        kms.append(ctx.last_kernel_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    kernel_ms = sum(kms) / len(kms)
    phased = args.precision != "bf16" and args.engine in (None, "mfma")
    engine = "phased" if phased else (args.engine or "pipelined")
    threads = args.threads or (512 if phased else 256 if engine == "valu" else 128)
    fl = flops_per_sample(inst.n_det, inst.n_lm, inst.n_t) * n
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    peak = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS,
            "bf16": BF16_PEAK_TFLOPS}[args.precision]
    out = {
        "metric": METRIC,
        "value": n * inst.n_t / (ms_step * 1e-3),
        "unit": "lnL evals/s (sample x time-bin)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "plain ILE at scale, one intrinsic point: 3 detectors, "
                               "21 modes (l=2..4), Q 16384 complex points at 16384 Hz, "
                               f"{n} prior samples, {inst.n_t} time bins",
                   "n_samples": n, "n_t": inst.n_t, "n_det": inst.n_det,
                   "n_lm": inst.n_lm, "precision": args.precision,
                   "engine": engine, "threads": threads},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": committed_traffic(args.precision, engine, threads),
                     "kernel": ("k_terms + k_contract_ph" if phased else "k_contract"),
                     "kernel_ms": kernel_ms, "flops_per_launch": fl},
        "result": {"ln_L_marg": res["ln_L_marg"], "n_eff": res["n_eff"],
                   "sigma_ln_L": res["sigma_ln_L"]},
    }
    ctx.close()
    out["precision_forms"] = None if args.no_forms else precision_forms(inst, n, seed, 3)
    out["mode_scaling"] = None if args.no_modes else mode_scaling_leg()
    out["latency"] = None if args.no_latency else latency_leg()
    out["harvest"] = None if args.no_harvest else harvest_leg(inst, n, seed)
    out["learned"] = None if args.no_learned else learned_leg()
    out["qvu"] = None if args.no_qvu else qvu_leg()
    out["rom"] = None if args.no_rom else rom_leg()
    out["batched"] = None if args.no_batched else batched_leg()
    out["reuse"] = None if args.no_reuse else reuse_leg()
    out["combined"] = None if args.no_combined else combined_leg(args.combined_points,
                                                                 first=args.combined_first)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, n_total, seed)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
