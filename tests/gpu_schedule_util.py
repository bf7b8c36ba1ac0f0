"""GPU side of the whole-schedule parity checks (test_gpu_schedule.py, test_gpu_batched.py): a
study stepped through the public entry points iteration by iteration, the lockstep comparison
with the oracle on the GPU's own state, and the comparison of independent schedules."""
import dataclasses

import numpy as np
import torch

import oracle
from paper_1803_10045_amd import kcs
from kcs_testutil import decision_bound, gpu_accepted, kcs_objects, oracle_decisions, rel_l2

DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.cpu().numpy().astype(np.float64)


class GpuSchedule:
    """GPU state of one study stepped through the public entry points."""

    def __init__(self, st, eta):
        self.st = st
        self.g, self.f, self.k, self.p, lm = kcs_objects(st)
        self.lm = dataclasses.replace(lm, eta=eta)
        self.one = dataclasses.replace(self.lm, n_iter=1)
        g, M = self.g, st.frames.M
        self.sino = dev(st.sino)
        self.x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
        self.params = torch.empty((self.k.n_maps, g.nz, g.ny, g.nx), device=DEV)
        self.lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
        self.work = kcs.alloc_workspace(g, M, st.cfg.Q, DEV)
        kcs.kcs_init_state(g, self.f, self.sino, oracle.initial_maps(st), self.x, self.params, self.lam, self.work)
        self.init = (self.x.clone(), self.params.clone(), self.lam.clone())

    def osl_pass(self, s):
        p = dataclasses.replace(self.p, kp_on=bool(self.p.kp_on and s > 0))
        for q in range(self.st.cfg.Q):
            kcs.kcs_osl_update(self.g, self.f, self.k, p, self.sino, self.params, q, self.st.cfg.Q, self.x, self.work)
        self.lam.zero_()  # every sweep's fit starts its damping afresh

    def lm_iteration(self):
        kcs.kcs_lm_fit(self.g, self.f, self.k, self.p, self.one, self.x, self.params, self.lam, self.work)

    def sweeps_through_icm(self, n_sweeps):
        """The same schedule through kcs_icm_sweep from the same initial state (host x, params,
        lam): the fit carries its normal equations between iterations, which must round exactly
        like the single-iteration calls."""
        return self.full_size_sweeps(self.g.nz, n_sweeps)

    def full_size_sweeps(self, nz_full, n_sweeps):
        """kcs_icm_sweep at nz_full planes, plane z holding the sampled plane z mod nz (sinogram and
        initial state); returns host (x, params, lam) of the full study."""
        st, g = self.st, self.g
        rep = torch.arange(nz_full, device=DEV) % g.nz
        gf = dataclasses.replace(g, nz=nz_full)
        sino = self.sino[rep].contiguous()
        x = self.init[0][rep].contiguous()
        params = self.init[1][:, rep].contiguous()
        lam = self.init[2][rep].contiguous()
        work = kcs.alloc_workspace(gf, st.frames.M, st.cfg.Q, DEV)
        for s in range(n_sweeps):
            kcs.kcs_icm_sweep(gf, self.f, self.k, self.p, self.lm, sino, st.cfg.Q, s, x, params, lam, work)
        torch.cuda.synchronize()
        return x.cpu().numpy(), params.cpu().numpy(), lam.cpu().numpy()


def assert_same_as_icm_sweeps(run, n_sweeps):
    ix, ip, il = run.sweeps_through_icm(n_sweeps)
    assert np.array_equal(ix, run.x.cpu().numpy())
    assert np.array_equal(ip, run.params.cpu().numpy())
    assert np.array_equal(il, run.lam.cpu().numpy())


def run_gpu(st, n_sweeps, eta, lockstep, osl_lockstep_sweeps=None):
    """The GPU schedule iteration by iteration; with `lockstep` the oracle repeats every LM
    iteration on the GPU's state, and every OSL pass of the first `osl_lockstep_sweeps` sweeps
    (all by default).  Returns the GPU run, its damping after every iteration, its image after
    every sweep and the lockstep statistics (LM decisions and maps, worst OSL pass)."""
    run = GpuSchedule(st, eta)
    opt = dataclasses.replace(st.lm, eta=eta, n_iter=1)
    sino = st.sino.astype(np.float64)
    lams, xs = [], []
    n_diff = n_dec = 0
    worst = 0.0
    map_err = 0.0
    osl_err = 0.0
    n_osl = n_sweeps if osl_lockstep_sweeps is None else osl_lockstep_sweeps
    for s in range(n_sweeps):
        if lockstep and s < n_osl:
            ox, op = host(run.x), host(run.params)
            kp = bool(st.prior.kp_on and s > 0)
            F = oracle.model_tac(op.reshape(len(op), -1).T, st.frames.t0, st.frames.t1, st.kin).reshape(ox.shape) if kp else None
            for q in range(st.cfg.Q):
                ox = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, sino, op, ox, q, st.cfg.Q, kp, None, F)
        run.osl_pass(s)
        x = host(run.x)
        xs.append(x.astype(np.float32))
        if lockstep and s < n_osl:
            osl_err = max(osl_err, rel_l2(x, ox))
        for it in range(st.lm.n_iter):
            if lockstep:
                p0, l0 = host(run.params), host(run.lam)
            run.lm_iteration()
            lams.append(run.lam.cpu().numpy())
            if lockstep:
                p1, l1 = host(run.params), lams[-1].astype(np.float64)
                op, _, acc, phi0, phi1, used = oracle_decisions(st, opt, x, p0, l0)
                differ = gpu_accepted(l0, l1, used, opt.lam_min) != acc
                n_diff += int(differ.sum())
                n_dec += differ.size
                if differ.any():
                    ratio = np.abs(phi1 - phi0 + eta * phi0) / decision_bound(x, phi0, phi1)
                    worst = max(worst, float(ratio[differ].max()))
                same = ~differ
                map_err = max(map_err, max(rel_l2(p1[i][same], op[i][same]) for i in range(len(op))))
    torch.cuda.synchronize()
    return run, np.stack(lams), np.stack(xs), (n_diff, n_dec, worst, map_err, osl_err)


def check_lockstep(label, eta, stats, max_frac, osl_tol=1e-5):
    """Every differing decision unresolvable in FP32, agreeing voxels' maps within 1e-4 after an
    iteration, each OSL pass (all subsets) within osl_tol of the oracle's pass on the same state."""
    n_diff, n_dec, worst, map_err, osl_err = stats
    print(f"{label} eta={eta}: lockstep: OSL passes within {osl_err:.2e}; {n_diff} of {n_dec} MAP-LM decisions "
          f"differ from the oracle's on the same state, largest margin {worst:.3f} of the FP32 bound; maps of "
          f"agreeing voxels within {map_err:.2e}")
    assert worst <= 1.0
    assert n_diff <= max_frac * n_dec
    assert map_err < 1e-4
    assert osl_err < osl_tol


def check_independent(label, eta, st, gx, gp, ox, op, first, margin, bound, inherited, max_diverged,
                      image_tol=1e-3, margin_check=True):
    """The oracle's own schedule against the GPU's: the image within image_tol, the maps of the
    active voxels whose decisions all agreed within 1e-3, every first differing decision of a
    voxel's own within its bound (margin_check).  The fraction of active voxels that took another
    path is a measure of how far the near-ties cascade (a flipped fit moves the voxel's maps, the
    kinetics prior carries them into the image, the neighbours' states follow), not of the kernel's
    accuracy: it varies with the rounding of every step (e.g. 1.4 % to 2.3 % of the 128x128
    planes between two builds of the same kernels that round differently), and max_diverged only
    bounds it loosely."""
    act = (ox * (st.frames.t1 - st.frames.t0)).sum(axis=-1)
    mask = act >= 0.1 * act.max()
    diverged = first >= 0
    keep = mask & ~diverged
    ex = rel_l2(gx, ox)
    literal = [rel_l2(gp[i][mask], op[i][mask]) for i in range(len(op))]
    kept = [rel_l2(gp[i][keep], op[i][keep]) for i in range(len(op))]
    frac = float(diverged[mask].mean())
    own = diverged & ~inherited
    ratio = margin[own] / bound[own]
    print(f"{label} eta={eta}: image relL2 {ex:.2e}; maps over active voxels {['%.2e' % e for e in literal]}; over "
          f"voxels whose decisions all agreed {['%.2e' % e for e in kept]}; {int((diverged & mask).sum())} of "
          f"{int(mask.sum())} active voxels took another path ({int(own.sum())} voxels of all by a near-tie of "
          f"their own, at margins <= {ratio.max() if ratio.size else 0.0:.3f} of the bound; "
          f"{int((diverged & inherited).sum())} after a neighbour)")
    assert ex < image_tol
    assert max(kept) < 1e-3
    if margin_check:
        assert ratio.size == 0 or ratio.max() <= 1.0
    assert frac <= max_diverged




def gpu_fit_history(g, f, k, p, lm, x, params0, lam0):
    """A MAP-LM fit through kcs_lm_fit one iteration at a time (host arrays in, lambda recorded
    after every iteration), checked bit for bit against the same fit in one call.  Returns the
    final host (params, lam) and the lambda history (n_iter, ...)."""
    M = x.shape[-1]
    work = kcs.alloc_workspace(g, M, 0, DEV)
    xd = dev(x)
    one = dataclasses.replace(lm, n_iter=1)
    pd, ld = dev(params0), dev(lam0)
    hist = []
    for _ in range(lm.n_iter):
        kcs.kcs_lm_fit(g, f, k, p, one, xd, pd, ld, work)
        hist.append(ld.cpu().numpy())
    pf, lf = dev(params0), dev(lam0)
    kcs.kcs_lm_fit(g, f, k, p, lm, xd, pf, lf, work)
    torch.cuda.synchronize()
    assert torch.equal(pf, pd) and torch.equal(lf, ld), "a fit in one call must round like its iterations"
    return pd.cpu().numpy(), ld.cpu().numpy(), np.stack(hist)
