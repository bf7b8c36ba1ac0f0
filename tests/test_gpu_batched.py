"""GPU: batched plans (many uneven studies per launch) against the plain per-study calls.

The studies of a plan are independent, so each study's result must equal what kcs_icm_sweep
gives on that study alone (same kernels, same projector variant: identical up to rounding), the
captured graph must reproduce the eager plan, and three of the studies (the 64x64 slice and a
128x128 and a 172x172 study of the batch recipe) must match the FP64 oracle's schedules.
Fused multiply-adds are formed per source expression, so the table-driven kernels of a plan round
like the single-study ones: plan and plain loop agree bit for bit."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from gpu_schedule_util import check_independent, host, run_gpu
from kcs_testutil import kcs_objects, oracle_schedule_vs_gpu, rel_l2

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
        assert err == 0.0


def test_plan_graph_matches_eager_plan(batch):
    studies, ranges, ref = batch
    ds, desc = planned(studies, ranges, kcs.KCS_PLAN_GRAPH)
    assert "graph=yes" in desc
    for st, a, b in zip(studies, ds, ref):
        err = state_errors(a, b)
        print(f"{st.cfg.name}: graph plan vs plain relL2 {err:.2e}")
        assert err == 0.0


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


def test_autotuned_plan_equals_plain_calls():
    """The plan autotuner times the projector variants per study shape and keeps the fastest for
    that shape for the rest of the process: plain calls on studies of a tuned shape use the same
    variant, so they reproduce the autotuned plan bit for bit.  The shapes here occur in no other
    test (a 150x150 plane is large enough for the tiled variants to compete)."""
    cfgs = [inputs.StudyConfig("tune_80x80x2", 80, 80, 2, 3.0, 3.0, 100, 80, 3.0, 8e5, 0.1, Q=5, n_sweeps=3,
                               phantom="brain", n_lesions=2, seed=51),
            inputs.StudyConfig("tune_150x150x2", 150, 150, 2, 2.0, 2.0, 195, 150, 2.0, 8e5, 0.1, Q=6, n_sweeps=2,
                               phantom="brain", n_lesions=2, seed=52)]
    studies = [oracle.make_study(c) for c in cfgs]
    ranges = [(0, c.n_sweeps) for c in cfgs]
    ds = [device_state(st) for st in studies]
    plan = kcs.kcs_plan_create([as_study(d, st.cfg.Q, r) for d, st, r in zip(ds, studies, ranges)],
                               kcs.KCS_PLAN_AUTOTUNE | kcs.KCS_PLAN_GRAPH)
    print(kcs.kcs_plan_describe(plan))
    kcs.kcs_plan_run(plan)
    torch.cuda.synchronize()
    kcs.kcs_plan_destroy(plan)
    ref = plain_loop(studies, ranges)
    for st, a, b in zip(studies, ds, ref):
        err = state_errors(a, b)
        print(f"{st.cfg.name}: autotuned plan vs plain calls relL2 {err:.2e}")
        assert err == 0.0


def test_plan_studies_match_oracle(batch):
    """The 64x64 slice and the two batch-recipe studies (128x128x3, 172x172x2: the latter takes the
    tiled projector), each after its sweeps in the plan, against the FP64 oracle.  The plan's
    result must equal, bit for bit, the same schedule stepped one MAP-LM iteration at a time, whose
    decisions are then compared with the oracle's iteration by iteration: the image over all voxels
    and the maps over the active voxels whose every decision agreed must be within 1e-3, at most
    2 % of them on another path, each of those first taken at a near-tie (FP32 bound); the maps over
    all active voxels are reported."""
    studies, ranges, _ = batch
    ds, _ = planned(studies, ranges, kcs.KCS_PLAN_GRAPH)
    for k in (0, 1, 2):
        st, (s0, s1) = studies[k], ranges[k]
        assert s0 == 0
        run, lams, xs, _ = run_gpu(st, s1, st.lm.eta, lockstep=False)
        for name in ("x", "params", "lam"):
            assert torch.equal(ds[k][name], getattr(run, name)), name
        ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, s1, st.lm.eta, lams, xs)
        check_independent(f"batched {st.cfg.name}, {s1} sweeps,", st.lm.eta, st, host(run.x), host(run.params), ox, op,
                          first, margin, bound, inherited, max_diverged=0.02)


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
        assert err == 0.0
