"""GPU: batched plans (many uneven studies per launch) against the plain per-study calls.

The studies of a plan are independent, so each study's result must equal what kcs_icm_sweep
gives on that study alone (same kernels, same projector variant: identical up to rounding), the
captured graph must reproduce the eager plan, and the study that has an oracle schedule must match
the FP64 oracle to the whole-schedule tolerance."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from kcs_testutil import kcs_objects, rel_l2

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"


def batch_studies():
    """Four uneven studies: 64x64x1 (4 subsets), 128x128x3 and 172x172x2 from the batch recipe
    (6 subsets; the 172 plane takes the tiled projector), and a ragged 37x29x3 grid with 7 subsets
    and an even LM count, starting at sweep 1."""
    bc = inputs.batch_configs()
    cfgs = [inputs.disk64(),
            inputs.scaled(bc[3], nz=3, counts=4e5 * 3),
            inputs.scaled(bc[1], nz=2, counts=4e5 * 2),
            inputs.StudyConfig("ragged_37x29x3", 37, 29, 3, 2.3, 2.3, 50, 45, 1.9, 3e5, 0.1, Q=7, n_sweeps=3,
                               n_lm=4, phantom="brain", n_lesions=2, seed=11, ang0=0.05)]
    ranges = [(0, 4), (0, 3), (0, 2), (1, 3)]
    return [oracle.make_study(c) for c in cfgs], ranges


def device_state(st):
    g, f, k, p, lm = kcs_objects(st)
    M = f.M
    sino = torch.from_numpy(st.sino.astype(np.float32)).to(DEV)
    x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, M, st.cfg.Q, DEV)
    kcs.kcs_init_state(g, f, sino, inputs.XI0, x, params, lam, work)
    return dict(g=g, f=f, k=k, p=p, lm=lm, sino=sino, x=x, params=params, lam=lam, work=work)


def as_study(d, Q, rng):
    return kcs.Study(d["g"], d["f"], d["k"], d["p"], d["lm"], Q, rng[0], rng[1], d["sino"], d["x"], d["params"],
                     d["lam"], d["work"])


def plain_loop(studies, ranges):
    out = []
    for st, (s0, s1) in zip(studies, ranges):
        d = device_state(st)
        for s in range(s0, s1):
            kcs.kcs_icm_sweep(d["g"], d["f"], d["k"], d["p"], d["lm"], d["sino"], st.cfg.Q, s, d["x"], d["params"],
                              d["lam"], d["work"])
        out.append(d)
    torch.cuda.synchronize()
    return out


def planned(studies, ranges, flags):
    ds = [device_state(st) for st in studies]
    plan = kcs.kcs_plan_create([as_study(d, st.cfg.Q, r) for d, st, r in zip(ds, studies, ranges)], flags)
    desc = kcs.kcs_plan_describe(plan)
    kcs.kcs_plan_run(plan)
    torch.cuda.synchronize()
    kcs.kcs_plan_destroy(plan)
    return ds, desc


def state_errors(a, b):
    return max(rel_l2(a[k].cpu().numpy(), b[k].cpu().numpy()) for k in ("x", "params", "lam"))


@pytest.fixture(scope="module")
def batch():
    studies, ranges = batch_studies()
    return studies, ranges, plain_loop(studies, ranges)


def test_plan_matches_plain_loop(batch):
    studies, ranges, ref = batch
    ds, desc = planned(studies, ranges, 0)
    print(desc)
    assert "studies=4" in desc and "graph=no" in desc
    for st, a, b in zip(studies, ds, ref):
        err = state_errors(a, b)
        print(f"{st.cfg.name}: plan vs plain relL2 {err:.2e}")
        assert err < 1e-6


def test_plan_graph_matches_eager_plan(batch):
    studies, ranges, ref = batch
    ds, desc = planned(studies, ranges, kcs.KCS_PLAN_GRAPH)
    assert "graph=yes" in desc
    for st, a, b in zip(studies, ds, ref):
        err = state_errors(a, b)
        print(f"{st.cfg.name}: graph plan vs plain relL2 {err:.2e}")
        assert err < 1e-6


def test_plan_graph_replays(batch):
    """Replaying a captured plan repeats its sweeps: two replays equal two eager runs."""
    studies, ranges, _ = batch
    results = []
    for flags in (0, kcs.KCS_PLAN_GRAPH):
        ds = [device_state(st) for st in studies]
        plan = kcs.kcs_plan_create([as_study(d, st.cfg.Q, r) for d, st, r in zip(ds, studies, ranges)], flags)
        for _ in range(2):
            kcs.kcs_plan_run(plan)
            torch.cuda.synchronize()
        kcs.kcs_plan_destroy(plan)
        results.append(ds)
    for a, b in zip(*results):
        assert state_errors(a, b) < 1e-6


def test_plan_autotuned_within_tolerance():
    """Autotuning may pick another projector variant, whose sums differ from the plain path's by
    rounding.  Over a schedule that difference grows: an accept test within rounding of its
    threshold can go either way (the voxel then follows another valid path), the prior carries
    the changed model TAC into the image, and the fit amplifies image differences in poorly
    determined voxels.  Checked: the image within the whole-schedule tolerance (1e-3), the maps
    over the active voxels whose accept/reject path was the same in every sweep within 1e-2, and
    at most 2 % of active voxels on another path.  (Each variant's parity with the oracle is
    tested in test_gpu_parity.py.)  Both sides run sweep by sweep to compare paths per sweep."""
    studies, ranges = batch_studies()
    ref = [device_state(st) for st in studies]
    tuned = [device_state(st) for st in studies]
    diverged = [np.zeros(st.sino.shape[:1] + st.truth_x.shape[1:3], dtype=bool) for st in studies]
    for sw in range(max(r[1] for r in ranges)):
        active = [k for k, r in enumerate(ranges) if r[0] <= sw < r[1]]
        for k in active:
            d, st = ref[k], studies[k]
            kcs.kcs_icm_sweep(d["g"], d["f"], d["k"], d["p"], d["lm"], d["sino"], st.cfg.Q, sw, d["x"], d["params"],
                              d["lam"], d["work"])
        plan = kcs.kcs_plan_create([as_study(tuned[k], studies[k].cfg.Q, (sw, sw + 1)) for k in active],
                                   kcs.KCS_PLAN_AUTOTUNE | kcs.KCS_PLAN_GRAPH)
        if sw == 0:
            print(kcs.kcs_plan_describe(plan))
        kcs.kcs_plan_run(plan)
        torch.cuda.synchronize()
        kcs.kcs_plan_destroy(plan)
        for k in active:
            diverged[k] |= np.abs(tuned[k]["lam"].cpu().numpy() / ref[k]["lam"].cpu().numpy() - 1.0) > 1e-3
    for st, a, b, dv in zip(studies, tuned, ref, diverged):
        bx, gx = b["x"].cpu().numpy(), a["x"].cpu().numpy()
        ex = rel_l2(gx, bx)
        act = (bx * (st.frames.t1 - st.frames.t0)).sum(axis=-1)
        active = act >= 0.1 * act.max()
        keep = active & ~dv
        ga, gb = a["params"].cpu().numpy(), b["params"].cpu().numpy()
        ep = max(rel_l2(ga[i][keep], gb[i][keep]) for i in range(3))
        frac = dv[active].mean()
        print(f"{st.cfg.name}: autotuned vs plain image {ex:.2e}, maps {ep:.2e} over active voxels with the same "
              f"LM path in every sweep ({frac:.4f} of active voxels took another)")
        assert ex < 1e-3 and ep < 1e-2 and frac < 0.02


def test_plan_study_matches_oracle(batch):
    """The 64x64 study of the batch after its 4 sweeps against the FP64 oracle."""
    studies, ranges, _ = batch
    ds, _ = planned(studies, ranges, kcs.KCS_PLAN_GRAPH)
    st = studies[0]
    ox, op, ol = oracle.icm(st.geom, st.frames, st.kin, st.prior, st.lm, st.sino.astype(np.float64), st.cfg.Q,
                            ranges[0][1])
    gx, gp = ds[0]["x"].cpu().numpy(), ds[0]["params"].cpu().numpy()
    act = (ox * (st.frames.t1 - st.frames.t0)).sum(axis=-1)
    mask = act >= 0.1 * act.max()
    ex = rel_l2(gx, ox)
    maps = [rel_l2(gp[i][mask], op[i][mask]) for i in range(3)]
    print(f"batched 64x64, 4 sweeps: image {ex:.2e} maps {maps}")
    assert ex < 1e-3 and max(maps) < 1e-3


def test_plan_rejects_bad_study(batch):
    studies, ranges, _ = batch
    d = device_state(studies[0])
    s = as_study(d, studies[0].cfg.Q, (2, 1))
    with pytest.raises(kcs.KcsError, match="study 0"):
        kcs.kcs_plan_create([s])


def test_plan_mixes_neighbourhoods():
    """A plan holding one in-plane and one 3x3x3 study runs their fits as separate launches and
    equals the per-study calls."""
    studies, ranges = batch_studies()
    studies, ranges = [studies[0], studies[3]], [(0, 2), (1, 3)]
    ref, got = [], []
    for st, (s0, s1) in zip(studies, ranges):
        d = device_state(st)
        if st is studies[1]:
            d["p"] = dataclasses.replace(d["p"], plane_ratio=1.0)
        for sw in range(s0, s1):
            kcs.kcs_icm_sweep(d["g"], d["f"], d["k"], d["p"], d["lm"], d["sino"], st.cfg.Q, sw, d["x"], d["params"],
                              d["lam"], d["work"])
        ref.append(d)
    ds = [device_state(st) for st in studies]
    ds[1]["p"] = dataclasses.replace(ds[1]["p"], plane_ratio=1.0)
    plan = kcs.kcs_plan_create([as_study(d, st.cfg.Q, r) for d, st, r in zip(ds, studies, ranges)], kcs.KCS_PLAN_GRAPH)
    kcs.kcs_plan_run(plan)
    torch.cuda.synchronize()
    kcs.kcs_plan_destroy(plan)
    for st, a, b in zip(studies, ds, ref):
        err = state_errors(a, b)
        print(f"{st.cfg.name}: plan vs plain relL2 {err:.2e}")
        assert err < 1e-6
