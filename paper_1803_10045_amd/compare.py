"""The paper's method comparison on synthetic data (Sec. III-B), run through the batched engine.

Three reconstructions of the same noisy dynamic data:

* INDIRECT: frame-by-frame OS-EM (no kinetics-derived prior) with a voxel-wise fit of the kinetic
  model to the images (no spatial prior);
* DIRECT: OS-MAP-OSL-KP (Eq. 2-3) alternating with the fit, without the spatial prior of the fit
  (beta_h = 0);
* KCS DIRECT: the same with the Huber prior on the maps' spatial differences (Eq. 5-7).

All three are ICM sweeps of the library with different prior settings: INDIRECT turns the
kinetics-derived prior off in every sweep, so each sweep's fit only follows the OS-EM image (its
maps after the last sweep are the post-fit of the final image, warm-started from the previous
sweeps).  Many noise realizations of one study run as the studies of one plan per sweep, and
after the recorded sweeps the bias and the standard deviation of the fitted maps and of the net
uptake rate K_i are taken per region against the truth (the bias/variance analysis of the
simulation).

The statistics are plain NumPy; every reconstruction step runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Iterable, List, Sequence

import numpy as np

from . import inputs, kcs

METHODS = ("indirect", "direct", "kcs")


def method_prior(prior: kcs.Prior, method: str, beta_h: float) -> kcs.Prior:
    """Prior settings of a method: INDIRECT no kinetics-derived prior and no spatial prior,
    DIRECT the kinetics-derived prior only, KCS both (spatial weight beta_h)."""
    if method == "indirect":
        return dataclasses.replace(prior, kp_on=False, beta_h=0.0)
    if method == "direct":
        return dataclasses.replace(prior, kp_on=True, beta_h=0.0)
    if method == "kcs":
        return dataclasses.replace(prior, kp_on=True, beta_h=beta_h)
    raise ValueError(method)


def synthesize_truth(cfg: inputs.StudyConfig, dev):
    """Noise-free data of the ring phantom: (geometry, frames, kinetics, base prior, LM options,
    expected counts ybar [nz][n_ang][n_bin][M] on the device, true maps (3, nz, ny, nx), region
    labels).  The tissue TACs are the model's; the blood square carries the plasma input itself
    (the model TAC at K1 = k2 = k3 = 0 divided by the blood fraction).  Counts are scaled to
    cfg.counts, with a flat background of cfg.bg_frac of them."""
    import torch

    g = kcs.Geometry.from_config(cfg)
    t0, t1 = inputs.frame_times(cfg.frame_blocks)
    dt = t1 - t0
    M = len(t0)
    kin = kcs.Kinetics(**inputs.FENG, vb=inputs.VB)
    maps, mask = inputs.phantom_maps(cfg)
    labels = inputs.ring_labels(cfg)
    N = g.n_vox
    p = torch.from_numpy(maps.reshape(3, N).astype(np.float32)).to(dev)
    x = torch.empty((N, M), device=dev)
    unit = kcs.Frames(t0, t1, np.ones(M), np.zeros(M))
    kcs.kcs_model_tac(unit, kin, p, x, None, kcs.alloc_workspace(None, M, 0, dev))
    lab = torch.from_numpy(labels.reshape(N)).to(dev)
    x[lab == 1] /= inputs.VB
    x[lab == 0] = 0.0
    x = x.view(g.nz, g.ny, g.nx, M)
    y = torch.empty((g.nz, g.n_ang, g.n_bin, M), device=dev)
    kcs.kcs_project(g, unit, x, 0, 1, y)
    total = float((y.view(-1, M).sum(dim=0, dtype=torch.float64).cpu().numpy() * dt).sum())
    c = cfg.counts / total
    E = c * dt
    r = cfg.bg_frac * cfg.counts * (dt / dt.sum()) / (cfg.n_ang * cfg.n_bin * cfg.nz)
    y.mul_(torch.from_numpy(E.astype(np.float32)).to(dev)).add_(torch.from_numpy(r.astype(np.float32)).to(dev))
    f = kcs.Frames(t0, t1, E, r)
    delta = inputs.huber_delta(maps, labels > 0)
    prior = kcs.Prior(inputs.BETA_KP, 1e-4 * peak_input(), cfg.beta_h, (delta,) * 3, True)
    lm = kcs.LMOptions(cfg.n_lm, inputs.LM_TAU, inputs.LM_LAM_MIN, inputs.LM_LAM_MAX, inputs.LM_LO, inputs.LM_HI,
                       inputs.LM_ETA)
    return g, f, kin, prior, lm, y, maps, labels


def peak_input() -> float:
    """max_t Cp(t) of the Feng input (the floor eps_F of the OSL-KP denominator is 1e-4 of it),
    by bounded minimisation of -Cp over the first two minutes, where its peak lies."""
    from scipy.optimize import minimize_scalar

    k = inputs.FENG

    def neg_cp(t):
        return -((k["A1"] * t - k["A2"] - k["A3"]) * np.exp(k["l1"] * t) + k["A2"] * np.exp(k["l2"] * t)
                 + k["A3"] * np.exp(k["l3"] * t))

    return -minimize_scalar(neg_cp, bounds=(0.0, 2.0), method="bounded", options=dict(xatol=1e-10)).fun


def realization(ybar, seed: int):
    """One Poisson realization of the expected counts (device, seeded)."""
    import torch

    gen = torch.Generator(device=ybar.device)
    gen.manual_seed(int(seed))
    return torch.poisson(ybar, generator=gen)


def run_method(g, f, kin, prior, lm, sinos: Sequence, Q: int, n_sweeps: int, record: Iterable[int], dev,
               flags: int = 0) -> Dict[int, np.ndarray]:
    """ICM sweeps of every realization in `sinos` as one plan per sweep (run once each, so not
    captured as a graph unless `flags` asks for it).  Returns, for each sweep
    count in `record`, the maps of all realizations (R, 3, nz, ny, nx) and their K_i (R, nz, ny, nx)
    stacked as (R, 4, nz, ny, nx)."""
    import torch

    M = f.M
    record = set(record)
    states = []
    for s in sinos:
        x = torch.empty((g.nz, g.ny, g.nx, M), device=dev)
        params = torch.empty((3, g.nz, g.ny, g.nx), device=dev)
        lam = torch.empty((g.nz, g.ny, g.nx), device=dev)
        work = kcs.alloc_workspace(g, M, Q, dev)
        kcs.kcs_init_state(g, f, s, inputs.XI0, x, params, lam, work)
        states.append((s, x, params, lam, work))
    ki = torch.empty((len(states), g.nz, g.ny, g.nx), device=dev)
    out = {}
    for sweep in range(n_sweeps):
        studies = [kcs.Study(g, f, kin, prior, lm, Q, sweep, sweep + 1, s, x, params, lam, work)
                   for s, x, params, lam, work in states]
        plan = kcs.kcs_plan_create(studies, flags)
        kcs.kcs_plan_run(plan)
        kcs.kcs_plan_destroy(plan)
        if sweep + 1 in record:
            for k, st in enumerate(states):
                kcs.kcs_ki_map(st[2], ki[k])
            torch.cuda.synchronize()
            maps = torch.stack([st[2] for st in states]).cpu().numpy()
            out[sweep + 1] = np.concatenate([maps, ki.cpu().numpy()[:, None]], axis=1)
    return out


def roi_stats(est: np.ndarray, truth: np.ndarray, region: np.ndarray) -> Dict[str, float]:
    """Bias and noise of one parameter over a region, in % of its true value (constant on the
    region): bias = |mean over the region of the realization-mean - truth| / truth,
    std = mean over the region of the across-realization standard deviation / truth.
    est: (R, ...) estimates, truth: (...) true values, region: (...) boolean."""
    t = float(np.mean(truth[region]))
    mean_v = est.mean(axis=0)[region]
    std_v = est.std(axis=0, ddof=1)[region] if est.shape[0] > 1 else np.zeros_like(mean_v)
    return {"bias_pct": 100.0 * abs(float(mean_v.mean()) - t) / t, "std_pct": 100.0 * float(std_v.mean()) / t}


def true_ki(maps: np.ndarray) -> np.ndarray:
    """K_i of the true maps, K1 k3 / (k2 + k3), and K1 where k2 + k3 = 0 (as kcs_ki_map)."""
    a = maps[1] + maps[2]
    return np.where(a > 0, maps[0] * maps[2] / np.where(a > 0, a, 1.0), maps[0])


def summarize(results: Dict[int, np.ndarray], maps: np.ndarray, labels: np.ndarray) -> List[dict]:
    """Rows (sweeps, region, parameter, bias %, std %) over the three tissue regions for K1 and K_i."""
    truth = {"K1": maps[0], "Ki": true_ki(maps)}
    rows = []
    for sweeps, est in sorted(results.items()):
        for reg in (2, 3, 4):
            region = labels == reg
            for name, k in (("K1", 0), ("Ki", 3)):
                st = roi_stats(est[:, k], truth[name], region)
                rows.append({"sweeps": sweeps, "region": inputs.RING_REGIONS[reg], "param": name,
                             "bias_pct": round(st["bias_pct"], 3), "std_pct": round(st["std_pct"], 3)})
    return rows
