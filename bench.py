#!/usr/bin/env python3
"""Benchmark of the kinetic compressive sensing hot path on one MI355X.

A step is one ICM sweep over one synthetic study: OS-MAP-OSL-KP over all subsets (forward
projection with the measured/expected ratio, gather back projection fused with the OSL update
and the kinetics-derived prior) followed by the synchronous MAP-LM iterations.  The default
workload is the clinical-scale study: 344x344x127 voxels (2.09 mm), 252 angles x 344 bins,
24 frames over 40 min, 21 subsets, 5 LM iterations, 3e8 counts + 15 % background.

Inputs are synthesised on the device (phantom maps from the seeded generator, activity from
kcs_model_tac, expected counts from kcs_project, Poisson draws) and are resident in HBM before
the timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def synthesize(cfg, dev, seed_offset=0, phantom=None, plane_ratio=0.0, correction=False):
    """Measured sinogram and study constants for `cfg`, built with the HIP library (`phantom`:
    the (maps, mask) of inputs.phantom_maps(cfg), if already computed; `correction`: a head-sized
    water cylinder's attenuation times detector efficiencies in the system matrix)."""
    import numpy as np
    import torch

    from paper_1803_10045_amd import inputs, kcs

    g = kcs.Geometry.from_config(cfg)
    if correction:
        import dataclasses
        mult = inputs.correction_sinogram(cfg.nz, cfg.n_ang, cfg.n_bin, cfg.bin_mm, 100.0, seed=cfg.seed)
        g = dataclasses.replace(g, mult=torch.from_numpy(mult).to(dev))
    t0, t1 = inputs.frame_times()
    dt = t1 - t0
    M = len(t0)
    kin = kcs.Kinetics(**inputs.FENG, vb=inputs.VB)
    maps, mask = inputs.phantom_maps(cfg) if phantom is None else phantom
    delta = inputs.huber_delta(maps, mask)
    N = g.n_vox
    p = torch.from_numpy(maps.reshape(3, N).astype(np.float32)).to(dev)
    m = torch.from_numpy(mask.reshape(N)).to(dev)
    p[:, ~m] = torch.tensor(inputs.XI0, dtype=torch.float32, device=dev)[:, None]  # any valid triple
    x = torch.empty((N, M), device=dev)
    work = kcs.alloc_workspace(None, M, 0, dev)
    kcs.kcs_model_tac(kcs.Frames(t0, t1, np.ones(M), np.zeros(M)), kin, p, x, None, work)
    x[~m] = 0.0
    x = x.view(g.nz, g.ny, g.nx, M)
    del p
    unit = kcs.Frames(t0, t1, np.ones(M), np.zeros(M))
    y = torch.empty((g.nz, g.n_ang, g.n_bin, M), device=dev)
    kcs.kcs_project(g, unit, x, 0, 1, y)
    per_frame = y.view(-1, M).sum(dim=0, dtype=torch.float64).cpu().numpy()
    total = float((per_frame * dt).sum())
    c = cfg.counts / total
    E = c * dt
    r = cfg.bg_frac * cfg.counts * (dt / dt.sum()) / (cfg.n_ang * cfg.n_bin * cfg.nz)
    y.mul_(torch.from_numpy(E.astype(np.float32)).to(dev)).add_(torch.from_numpy(r.astype(np.float32)).to(dev))
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg.seed + seed_offset)
    sino = torch.poisson(y, generator=gen)
    del y, x
    f = kcs.Frames(t0, t1, E, r)
    from scipy.optimize import minimize_scalar  # only for the peak of the input function
    cp = lambda t: -((inputs.FENG["A1"] * t - inputs.FENG["A2"] - inputs.FENG["A3"]) * np.exp(inputs.FENG["l1"] * t)
                     + inputs.FENG["A2"] * np.exp(inputs.FENG["l2"] * t) + inputs.FENG["A3"] * np.exp(inputs.FENG["l3"] * t))
    peak = -minimize_scalar(cp, bounds=(0.0, 2.0), method="bounded", options=dict(xatol=1e-10)).fun
    prior = kcs.Prior(inputs.BETA_KP, 1e-4 * peak, cfg.beta_h, (delta,) * 3, True, plane_ratio)
    lm = kcs.LMOptions(cfg.n_lm, inputs.LM_TAU, inputs.LM_LAM_MIN, inputs.LM_LAM_MAX, inputs.LM_LO, inputs.LM_HI,
                       inputs.LM_ETA)
    return g, f, kin, prior, lm, sino


def algorithmic_bytes(g, M, Q):
    """Compulsory HBM bytes per launch of each kernel (FP32; model TAC and sensitivity on the fly).
    K-proj (ratio): reads image I and the subset's measured sinogram, writes the ratio.
    K-back (OSL): reads the ratio, the image and the 3 maps, writes the image.
    K-lm: reads image, maps and lambda, writes maps and lambda."""
    N = g.n_vox
    I = N * M * 4
    A_mean = g.n_ang / Q
    S_q = g.nz * A_mean * g.n_bin * M * 4
    return {"project": I + 2 * S_q, "osl": 2 * I + S_q + 12 * N, "lm": I + 32 * N}


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1803_10045_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(cfg_name, kind):
    """HBM bytes per launch of step `kind` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload (scaled by the copy reference), or None when there is none or the
    kernel sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"sweep_{cfg_name.split('_', 1)[1]}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    if blob.get("source") != kernel_source_hash():
        return None
    return blob.get("traffic_bytes_per_launch", {}).get(kind)


def counter_busy(cfg_name, kind):
    """Fraction of SIMD cycles in which step `kind`'s main kernel issues at least one VALU
    instruction (dual-issue cycles counted once), from the committed compute-counter summary of
    this workload, or None (missing, or kernel sources changed since)."""
    path = os.path.join(ROOT, "profiles", f"sweep_{cfg_name.split('_', 1)[1]}_compute_counters.md")
    if not os.path.exists(path):
        return None
    try:
        blob = json.loads(open(path).read().split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    if blob.get("source") != kernel_source_hash():
        return None
    return blob.get("valu_busy", {}).get(kind)


def cpu_baseline(cfg):
    """The FP64 oracle on a bounded sample of the same workload, extrapolated to one sweep."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from paper_1803_10045_amd import inputs

    sample = inputs.scaled(cfg, nz=1)
    st = oracle.make_study(sample)
    sino = st.sino.astype(np.float64)
    x, params, lam = oracle.initial_state(st.geom, st.frames, sino)
    params = np.broadcast_to(np.array(inputs.GRAY)[:, None, None, None], params.shape).copy()
    oracle.system_matrix(st.geom)  # build outside the timed part (geometry setup, not per sweep)
    n_sub = min(cfg.Q, 6)
    ny, nx = 128, 128
    y0, x0 = cfg.ny // 2 - ny // 2, cfg.nx // 2 - nx // 2
    xs = np.ascontiguousarray(st.truth_x[:, y0:y0 + ny, x0:x0 + nx])
    ps0 = np.ascontiguousarray(params[:, :, y0:y0 + ny, x0:x0 + nx])
    n_vox = cfg.nx * cfg.ny * cfg.nz

    def timed(threads):
        with threadpool_limits(threads):
            xx = x.copy()
            t = time.perf_counter()
            for q in range(n_sub):
                xx = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, sino, params, xx, q, cfg.Q, True)
            t_osl = (time.perf_counter() - t) / n_sub
            ps, ls = ps0.copy(), np.zeros((1, ny, nx))
            t = time.perf_counter()
            for _ in range(2):
                ps, ls = oracle.lm_iteration(st.frames, st.kin, st.prior, st.lm, xs, ps, ls)
            t_lm = (time.perf_counter() - t) / 2
        return t_osl, t_lm, cfg.nz * cfg.Q * t_osl + cfg.n_lm * n_vox * t_lm / (nx * ny)

    def sample(t_osl, t_lm, threads):
        return (f"{n_sub} OSL subset updates on one {cfg.nx}x{cfg.ny} plane ({t_osl:.2f} s each) and 2 MAP-LM "
                f"iterations on {nx * ny} voxels ({t_lm:.2f} s each), FP64, {threads} thread(s); extrapolated to "
                f"{cfg.nz} planes x {cfg.Q} subsets and {cfg.n_lm} iterations x {n_vox} voxels")

    t_osl, t_lm, sweep_s = timed(1)
    out = {"value": 1.0 / sweep_s, "unit": "sweeps/s", "cores": 1, "kind": "oracle", "sample": sample(t_osl, t_lm, 1)}
    # the same sample with every host core the process may use (the oracle's C model loop runs in
    # OpenMP threads, NumPy/SciPy in their thread pools; the sparse products stay single-threaded)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():  # the host's share of cores, where it is set
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    t_osl, t_lm, sweep_s = timed(cores)
    out["all_cores"] = {"value": 1.0 / sweep_s, "unit": "sweeps/s", "cores": cores, "sample": sample(t_osl, t_lm,
                                                                                                       cores)}
    return out


def run_batched(args):
    """The uneven batch: every study from its initial state through all its sweeps, once as the
    plain per-study loop of kcs_icm_sweep calls and once as one batched plan (graph-captured,
    projector variant autotuned per study shape, which the plain calls then share).  A step is one
    pass over the whole batch."""
    import torch

    from paper_1803_10045_amd import inputs, kcs

    dev = torch.device("cuda:0")
    cfgs = inputs.batch_configs()
    studies = []
    t = time.perf_counter()
    for cfg in cfgs:
        g, f, kin, prior, lm, sino = synthesize(cfg, dev)
        M = f.M
        x = torch.empty((g.nz, g.ny, g.nx, M), device=dev)
        params = torch.empty((3, g.nz, g.ny, g.nx), device=dev)
        lam = torch.empty((g.nz, g.ny, g.nx), device=dev)
        work = kcs.alloc_workspace(g, M, cfg.Q, dev)
        studies.append(kcs.Study(g, f, kin, prior, lm, cfg.Q, 0, cfg.n_sweeps, sino, x, params, lam, work))
    torch.cuda.synchronize()
    n_vox = sum(s.g.n_vox for s in studies)
    log(f"synthesised {len(studies)} studies ({n_vox / 1e6:.1f} M voxels) in {time.perf_counter() - t:.1f} s")

    def reset():
        for s in studies:
            kcs.kcs_init_state(s.g, s.f, s.sino, inputs.XI0, s.x, s.params, s.lam, s.work)

    def plain():
        for s in studies:
            for sw in range(s.sweep_begin, s.sweep_end):
                kcs.kcs_icm_sweep(s.g, s.f, s.k, s.p, s.lm, s.sino, s.Q, sw, s.x, s.params, s.lam, s.work)

    def timed_runs(run, label):
        for _ in range(args.warmup):
            reset()
            run()
        torch.cuda.synchronize()
        total = 0.0
        for _ in range(args.steps):
            reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            run()
            b.record()
            torch.cuda.synchronize()
            total += a.elapsed_time(b)
        log(f"{label}: {total / args.steps:.1f} ms per batch")
        return total / args.steps

    # the plan is created (and its projector variants tuned per study shape) first: the plain loop
    # then uses the same variant for each shape, so the two compute the same sums
    t = time.perf_counter()
    plan = kcs.kcs_plan_create(studies, kcs.KCS_PLAN_GRAPH | kcs.KCS_PLAN_AUTOTUNE)
    log(f"plan created in {time.perf_counter() - t:.2f} s: {kcs.kcs_plan_describe(plan)}")
    ms_plain = timed_runs(plain, "plain per-study loop")
    ref = [(s.x.clone(), s.params.clone()) for s in studies]
    ms_plan = timed_runs(lambda: kcs.kcs_plan_run(plan), "batched plan")
    err_x = max(float((s.x - r[0]).norm() / r[0].norm()) for s, r in zip(studies, ref))

    def map_err(s, r):  # each map over the voxels above 10 % of peak activity, as in the parity tests
        dt = torch.from_numpy(s.f.t1 - s.f.t0).float().to(dev)
        act = (r[0] * dt).sum(dim=-1)
        mask = act >= 0.1 * act.max()
        return max(float((s.params[i][mask] - r[1][i][mask]).norm() / r[1][i][mask].norm()) for i in range(3))

    err_p = max(map_err(s, r) for s, r in zip(studies, ref))
    desc = kcs.kcs_plan_describe(plan)
    kcs.kcs_plan_destroy(plan)
    n = len(studies)
    out = {
        "metric": "batched studies/s",
        "value": round(n / (ms_plan * 1e-3), 4),
        "unit": "studies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_plan, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantoms, closed-form FDG TACs, Poisson counts)",
        "config": {"workload": f"{n} uneven studies (8-127 planes, 128 or 172 matrix, 1.3x angles, 6 subsets, "
                               f"10 sweeps each, {n_vox} voxels in total)"},
        "plain_loop_studies_per_s": round(n / (ms_plain * 1e-3), 4),
        "speedup_vs_plain": round(ms_plain / ms_plan, 3),
        "max_rel_l2_vs_plain": {"image": err_x, "maps_active_voxels": err_p},
        "plan": desc,
    }
    print(json.dumps(out), flush=True)


def _phantom(cfg):
    import numpy as np

    from paper_1803_10045_amd import inputs
    maps, mask = inputs.phantom_maps(cfg)
    return maps.astype(np.float32), mask


def make_requests(n, rate, dev):
    """The seeded request stream with phantoms computed up front (host work that belongs to the
    arrival of a study, not to its service); each request's loader synthesises its sinogram on the
    device when it is admitted."""
    from concurrent.futures import ProcessPoolExecutor

    from paper_1803_10045_amd import inputs, kcs, serve

    stream = inputs.request_stream(n, rate if rate > 0 else 4.0)
    with ProcessPoolExecutor(max_workers=8) as pool:
        phantoms = list(pool.map(_phantom, [cfg for _, cfg in stream]))
    reqs = []
    for j, ((t, cfg), ph) in enumerate(zip(stream, phantoms)):
        g = kcs.Geometry.from_config(cfg)
        req = serve.Request(j, t if rate > 0 else 0.0, g, None, None, None, None, cfg.Q, cfg.n_sweeps, None,
                            inputs.XI0)

        def load(req=req, cfg=cfg, ph=ph):
            _, f, kin, prior, lm, sino = synthesize(cfg, dev, phantom=ph)
            req.f, req.k, req.p, req.lm = f, kin, prior, lm
            return sino

        req.load = load
        # constants that do not depend on the synthesised counts are known before loading
        t0, t1 = inputs.frame_times()
        req.f = kcs.Frames(t0, t1, t1 - t0, 0 * t0)
        reqs.append(req)
    return reqs


def run_serve(args):
    """The served workload: Poisson arrivals of mixed-size studies, continuous batching at sweep
    granularity under an HBM budget, against the plain per-study loop serving the same stream one
    study at a time.  Also a saturated run (all requests at t = 0) for capacity."""
    import torch

    from paper_1803_10045_amd import kcs, serve

    dev = torch.device("cuda:0")
    budget = int(args.budget_gb * 1e9)
    out_runs = {}
    total_bytes = None
    runs = [r.split("@") for r in args.serve_runs.split(",")]
    for mode, when in runs:
        label = mode
        rate = args.rate if when == "poisson" else 0.0
        t = time.perf_counter()
        reqs = make_requests(args.requests, rate, dev)
        log(f"{len(reqs)} requests prepared in {time.perf_counter() - t:.1f} s (rate {rate or 'all at once'})")
        if total_bytes is None:
            total_bytes = 0
            for r in reqs:
                nb = algorithmic_bytes(r.g, r.f.M, r.Q)
                total_bytes += r.n_sweeps * (r.Q * (nb["project"] + nb["osl"]) + 5 * nb["lm"])
        if mode.startswith("served"):
            # "served:N" runs at most N small-study ticks beside a large study's tick
            cap = int(mode.split(":")[1].split("/")[0]) if ":" in mode else args.small_beside_large
            ex = serve.GpuExecutor(dev, n_lanes=2)
            wait = args.small_wait
            if "/" in mode:  # "served:N/W": W seconds of small-study wait beside a large study
                mode, w = mode.split("/")
                wait = float(w)
            comp, _, makespan, ticks = serve.serve(reqs, budget, ex, log=log, small_in_flight_beside_large=cap,
                                                   small_wait_beside_large=wait, large_resident=args.large_resident)
            ex.close()
            extra = {"ticks": ticks, "small_in_flight_beside_large": cap, "small_wait_beside_large_s": wait,
                     "large_resident": args.large_resident}
        else:
            comp, _, makespan = serve.serve_serial(reqs, log=log)
            extra = {}
        lat = serve.latency_summary(comp)
        size_of = {r.rid: f"{r.g.nx}x{r.g.ny}x{r.g.nz}" for r in reqs}
        by_size = {k: serve.latency_summary([c for c in comp if size_of[c.rid] == k])
                   for k in sorted(set(size_of.values()), key=lambda k: int(k.split("x")[0]))}
        res = {"studies_per_s": round(len(comp) / makespan, 3), "makespan_s": round(makespan, 2), **lat,
               "hbm_frac": round(total_bytes / makespan / (HBM_PEAK_GBPS * 1e9), 4), **extra, "by_size": by_size,
               "largest": [(c.rid, round(c.arrival, 3), round(c.admitted, 3), round(c.finished, 3))
                           for c in comp if size_of[c.rid] == max(size_of.values(), key=lambda k: int(k.split("x")[0]))]}
        key = f"{label}@{rate}Hz" if rate > 0 else f"{label}@saturated"
        out_runs[key] = res
        log(f"{key}: {res}")
        torch.cuda.empty_cache()
    nominal = out_runs.get(f"served@{args.rate}Hz", {})
    cap = out_runs.get("served@saturated", {})
    out = {
        "metric": "served studies/s",
        "value": cap.get("studies_per_s"),
        "unit": "studies/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": round(1e3 / cap["studies_per_s"], 2) if cap else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantoms, closed-form FDG TACs, Poisson counts)",
        "config": {"workload": f"{args.requests} requests, Poisson arrivals at {args.rate}/s, sizes 64x64x1 / "
                               "128x128x47 / 172x172x64 / 344x344x127 weighted 0.4/0.3/0.2/0.1, "
                               f"HBM budget {args.budget_gb} GB"},
        "p50_latency_s": nominal.get("p50_s"),
        "p99_latency_s": nominal.get("p99_s"),
        "runs": out_runs,
    }
    print(json.dumps(out), flush=True)


def run_copy(args):
    """The HBM rates this GPU sustains, from the library's streaming kernels: a plain read (2 GiB
    into one partial sum per thread) and a plain copy (2 GiB read, 2 GiB written), each at the
    workgroup count that runs fastest.  These are the ceilings the bandwidth-bound kernels are
    compared with, and the copy is the reference of known size against which the HBM byte counters
    of a profiled run are scaled."""
    import torch

    from paper_1803_10045_amd import kcs

    nbytes = 2 << 30
    src = torch.ones(nbytes // 4, device="cuda:0")
    dst = torch.empty_like(src)
    sums = torch.empty(8192 * 256, device="cuda:0")
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"bytes_per_launch": nbytes}
    for kind, name, moved in ((0, "read", nbytes), (1, "copy", 2 * nbytes)):
        best = None
        for groups in (256, 512, 1024, 2048, 4096):
            kcs.kcs_stream_probe(kind, src, sums if kind == 0 else dst, groups)  # warm-up
            torch.cuda.synchronize()
            t0.record()
            for _ in range(args.steps):
                kcs.kcs_stream_probe(kind, src, sums if kind == 0 else dst, groups)
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / args.steps
            if best is None or ms < best[1]:
                best = (groups, ms)
        out[name] = {"workgroups": best[0], "avg_ms": round(best[1], 4),
                     "GBps": round(moved / best[1] / 1e6, 1)}
        log(f"stream {name}: {out[name]}")
    print(json.dumps(out), flush=True)


def run_ki(args):
    """K_i map (net uptake rate) over the maps of a study of the chosen configuration: 16 B per
    voxel (3 maps read, 1 written), timed with HIP events over `steps` launches."""
    import torch

    from paper_1803_10045_amd import inputs, kcs

    cfg = inputs.CONFIGS[args.config]()
    shape = (cfg.nz, cfg.ny, cfg.nx)
    g = torch.Generator(device="cpu").manual_seed(5)
    lo = torch.tensor(inputs.LM_LO).view(3, 1, 1, 1)
    hi = torch.tensor(inputs.LM_HI).view(3, 1, 1, 1)
    params = (lo + (hi - lo) * torch.rand((3,) + shape, generator=g)).to("cuda:0")
    ki = torch.empty(shape, device="cuda:0")
    kcs.kcs_ki_map(params, ki)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        kcs.kcs_ki_map(params, ki)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    n = ki.numel()
    gbps = 16 * n / ms / 1e6
    print(json.dumps({"metric": "K_i map GB/s", "value": round(gbps, 1), "unit": "GB/s", "voxels": n,
                      "avg_ms": round(ms, 4), "launches": args.steps, "alg_bytes_per_launch": 16 * n,
                      "hbm_frac": round(gbps / 8000.0, 4), "config": {"workload": cfg.name}}), flush=True)


def run_ssrb(args):
    """Single-slice rebinning of a span-1 acquisition of the mMR's 64 rings (ring differences up to
    60) with the headline sinogram (252 angles x 344 bins) and 4 frames into its 127 planes,
    timed with HIP events over `steps` launches.  Algorithmic bytes: every existing ring pair's
    sinogram read once and the planes written once."""
    import torch

    from paper_1803_10045_amd import kcs

    R, D, A, B, M = 64, 60, 252, 344, 4
    g = torch.Generator(device="cuda:0")
    g.manual_seed(9)
    y3d = torch.poisson(torch.full((2 * D + 1, R, A, B, M), 2.0, device="cuda:0"), generator=g)
    y2d = torch.empty((2 * R - 1, A, B, M), device="cuda:0")
    count = torch.empty(2 * R - 1, device="cuda:0")
    kcs.kcs_rebin_ssrb(R, D, y3d, y2d, count)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        kcs.kcs_rebin_ssrb(R, D, y3d, y2d, count)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    pairs = int(count.sum().item())
    nbytes = (pairs + 2 * R - 1) * A * B * M * 4
    gbps = nbytes / ms / 1e6
    print(json.dumps({"metric": "rebinning GB/s", "value": round(gbps, 1), "unit": "GB/s", "avg_ms": round(ms, 4),
                      "launches": args.steps, "alg_bytes_per_launch": nbytes, "hbm_frac": round(gbps / 8000.0, 4),
                      "config": {"workload": f"{R} rings, ring differences up to {D} ({pairs} ring pairs), "
                                             f"{A} angles x {B} bins, {M} frames -> {2 * R - 1} planes"}}), flush=True)


def run_compare(args):
    """The method comparison of the simulation on the ring phantom: INDIRECT, DIRECT and KCS DIRECT
    (for each spatial weight of `--beta-h`, decades apart) over `--realizations` noise
    realizations (one plan per sweep over all of them), bias and standard deviation of K1 and K_i
    per region after 2, 5 and `--sweeps` sweeps."""
    import torch

    from paper_1803_10045_amd import compare, inputs

    dev = torch.device("cuda:0")
    cfg = inputs.rings_config(128, nz=4)
    g, f, kin, prior, lm, ybar, maps, labels = compare.synthesize_truth(cfg, dev)
    R, S = args.realizations, args.sweeps
    record = sorted({2, 5, S} & set(range(1, S + 1)))
    betas = [float(b) for b in args.beta_h.split(",")]
    runs = [("indirect", 0.0), ("direct", 0.0)] + [("kcs", b) for b in betas]
    out = {}
    t_all = 0.0
    for method, beta in runs:
        sinos = [compare.realization(ybar, 1000 + r) for r in range(R)]  # the same realizations for every run
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = compare.run_method(g, f, kin, compare.method_prior(prior, method, beta), lm, sinos, cfg.Q, S, record,
                                 dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        t_all += dt
        key = method if method != "kcs" else f"kcs@beta_h={beta:g}"
        out[key] = {"seconds": round(dt, 3), "rows": compare.summarize(res, maps, labels)}
        log(f"{key}: {R} realizations x {S} sweeps in {dt:.2f} s")
        del sinos, res
    print(json.dumps({"metric": "comparison realization-sweeps/s", "value": round(len(runs) * R * S / t_all, 2),
                      "unit": "realization-sweeps/s", "realizations": R, "sweeps": S,
                      "config": {"workload": f"{cfg.name}: ring phantom (Table I tissue parameters, blood square), "
                                             f"{cfg.n_ang} angles x {cfg.n_bin} bins, 24 frames (Eq. 8 blocks), "
                                             f"{cfg.Q} subsets, {cfg.counts:.1e} counts"},
                      "methods": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--mode", default="sweep", choices=["sweep", "batched", "serve", "copy", "ki", "compare", "ssrb"])
    ap.add_argument("--realizations", type=int, default=32, help="compare mode: noise realizations per method")
    ap.add_argument("--sweeps", type=int, default=10, help="compare mode: ICM sweeps per realization")
    ap.add_argument("--beta-h", default="1e2,1e3,1e4,1e5", help="compare mode: KCS spatial weights (comma-separated)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--budget-gb", type=float, default=250.0)
    ap.add_argument("--small-beside-large", type=int, default=1,
                    help="serve mode: small-study ticks in flight beside a large study's tick")
    ap.add_argument("--small-wait", type=float, default=0.0,
                    help="serve mode: seconds a small study waits before its ticks run beside a large one")
    ap.add_argument("--large-resident", type=int, default=1,
                    help="serve mode: most large studies resident (admitted and loaded) at once (0: no limit)")
    ap.add_argument("--serve-runs", default="served@poisson,serial@poisson,served@saturated,serial@saturated",
                    help="comma-separated runs of the serve mode: served[:N[/W]]|serial @ poisson|saturated "
                         "(N: --small-beside-large, W: --small-wait)")
    ap.add_argument("--config", default="brain344", choices=["disk64", "brain128", "brain344"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--correction", action="store_true",
                    help="sweep mode: attenuation (head-sized water cylinder) x detector efficiencies in the model")
    ap.add_argument("--plane-ratio", type=float, default=0.0,
                    help="sweep mode: > 0 fits with the 3x3x3 Huber neighbourhood, planes this many pixel sides apart")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the ICM sweep shards by plane with no "
              "exchange, and runs on more than one GPU are not supported.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "serve":
        run_serve(args)
        return
    if args.mode == "copy":
        args.steps = 4 if args.steps is None else args.steps
        run_copy(args)
        return
    if args.mode == "compare":
        run_compare(args)
        return
    if args.mode == "ssrb":
        if args.steps is None:
            args.steps = 10
        run_ssrb(args)
        return
    if args.mode == "ki":
        args.steps = 20 if args.steps is None else args.steps
        run_ki(args)
        return
    if args.mode == "batched":
        args.steps = 2 if args.steps is None else args.steps
        args.warmup = 1 if args.warmup is None else args.warmup
        run_batched(args)
        return
    args.steps = 10 if args.steps is None else args.steps
    args.warmup = 2 if args.warmup is None else args.warmup

    import numpy as np
    import torch

    from paper_1803_10045_amd import inputs, kcs

    dev = torch.device("cuda:0")
    cfg = inputs.CONFIGS[args.config]()
    t = time.perf_counter()
    g, f, kin, prior, lm, sino = synthesize(cfg, dev, plane_ratio=args.plane_ratio, correction=args.correction)
    torch.cuda.synchronize()
    log(f"synthesised {cfg.name} in {time.perf_counter() - t:.1f} s; counts {float(sino.sum()):.3e}")
    M, Q = f.M, cfg.Q
    x = torch.empty((g.nz, g.ny, g.nx, M), device=dev)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=dev)
    lam = torch.empty((g.nz, g.ny, g.nx), device=dev)
    work = kcs.alloc_workspace(g, M, Q, dev)
    kcs.kcs_init_state(g, f, sino, inputs.XI0, x, params, lam, work)
    sweep = 0
    for _ in range(args.warmup):
        kcs.kcs_icm_sweep(g, f, kin, prior, lm, sino, Q, sweep, x, params, lam, work)
        sweep += 1
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} sweeps done")

    kcs.kcs_timing_enable(True)
    kcs.kcs_timing_collect()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        kcs.kcs_icm_sweep(g, f, kin, prior, lm, sino, Q, sweep, x, params, lam, work)
        sweep += 1
    stop.record()
    torch.cuda.synchronize()
    elapsed_ms = start.elapsed_time(stop)
    timing = kcs.kcs_timing_collect()
    kcs.kcs_timing_enable(False)
    log(f"timed {args.steps} sweeps: {elapsed_ms:.2f} ms")
    if not torch.isfinite(x).all() or not torch.isfinite(params).all():
        raise RuntimeError("non-finite values in the reconstruction")

    nbytes = algorithmic_bytes(g, M, Q)
    kernels = {}
    for kind in ("project", "osl", "lm"):
        ms, n = timing[kind]
        if n == 0:
            continue
        avg = ms / n
        gbps = nbytes[kind] / (avg * 1e-3) / 1e9
        kernels[kind] = {"launches": n, "avg_ms": round(avg, 4), "ms_per_sweep": round(ms / args.steps, 3),
                         "alg_bytes_per_launch": int(nbytes[kind]), "alg_GBps": round(gbps, 1),
                         "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4)}
        # counter-measured HBM traffic and VALU issue of the same kernel (committed rocprofv3
        # summaries, averaged over a sweep's launches; None once the kernel sources changed)
        tb = counter_traffic(cfg.name, kind)
        kernels[kind]["traffic_GBps"] = None if tb is None else round(tb / (avg * 1e-3) / 1e9, 1)
        kernels[kind]["valu_busy"] = counter_busy(cfg.name, kind)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_sweep"])
    traffic = counter_traffic(cfg.name, dom)
    roof = {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["alg_GBps"], "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": kernels[dom]["hbm_frac"],
            "traffic": None if traffic is None else round(traffic / (kernels[dom]["avg_ms"] * 1e-3) / 1e9, 1),
            "traffic_bytes_per_launch": traffic, "alg_bytes_per_launch": kernels[dom]["alg_bytes_per_launch"]}
    roof["valu_busy"] = counter_busy(cfg.name, dom)
    value = args.steps / (elapsed_ms * 1e-3)
    out = {
        "metric": "ICM sweeps/s",
        "value": round(value, 3),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantom, closed-form FDG TACs, Poisson counts)",
        "config": {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny}x{cfg.nz} voxels, {cfg.n_ang} angles x {cfg.n_bin} "
                               f"bins, {M} frames, {Q} subsets, {cfg.n_lm} MAP-LM iterations per sweep"
                               + (f", 3x3x3 Huber neighbourhood (planes {args.plane_ratio} pixel sides apart)"
                                  if args.plane_ratio > 0 else "")
                               + (", attenuation x efficiency correction sinogram" if args.correction else ""),
                   "counts": cfg.counts, "background": cfg.bg_frac},
        "roofline": roof,
        "kernels": kernels,
        "proj_backproj_GBps": {"project": kernels.get("project", {}).get("alg_GBps"),
                               "backproject_osl": kernels.get("osl", {}).get("alg_GBps")},
    }
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(cfg)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
