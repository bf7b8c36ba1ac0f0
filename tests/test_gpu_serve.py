"""GPU: the continuous-batching server.  Each study's result must be the same when it is served
in a mix of overlapping studies as when it runs alone through the plain per-study calls (relative
L2 within 1e-5; the kernels are shared, so in practice identical)."""
import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from gpu_schedule_util import check_independent, host, run_gpu
from kcs_testutil import kcs_objects, oracle_schedule_vs_gpu, rel_l2

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs, serve  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"


def small_stream():
    specs = [  # (matrix x, y, planes, angles, bins, subsets, sweeps, arrival s, seed)
        (64, 64, 1, 60, 64, 4, 4, 0.00, 21),
        (48, 40, 2, 50, 44, 5, 3, 0.00, 22),
        (40, 40, 3, 36, 40, 3, 6, 0.00, 23),
        (64, 64, 2, 72, 64, 6, 2, 0.00, 24),
        (32, 32, 1, 30, 32, 2, 5, 0.01, 25),
        (56, 56, 1, 48, 56, 4, 3, 0.02, 26),
    ]
    reqs = []
    for j, (nx, ny, nz, na, nb, Q, sw, t, seed) in enumerate(specs):
        cfg = inputs.StudyConfig(f"s{j}", nx, ny, nz, 3.0, 3.0, na, nb, 3.0, 3e5 * nz, 0.1, Q=Q, n_sweeps=sw,
                                 phantom="disk" if nz == 1 else "brain", n_lesions=2, seed=seed)
        st = oracle.make_study(cfg)
        g, f, k, p, lm = kcs_objects(st)
        sino = np.ascontiguousarray(st.sino, np.float32)
        req = serve.Request(j, t, g, f, k, p, lm, Q, sw, lambda h=sino: torch.from_numpy(h).to(DEV), inputs.XI0)
        req.cfg = cfg
        reqs.append(req)
    return reqs


def alone(r):
    sino = r.load()
    g, M = r.g, r.f.M
    x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, M, r.Q, DEV)
    kcs.kcs_init_state(g, r.f, sino, r.xi0, x, params, lam, work)
    for s in range(r.n_sweeps):
        kcs.kcs_icm_sweep(g, r.f, r.k, r.p, r.lm, sino, r.Q, s, x, params, lam, work)
    torch.cuda.synchronize()
    return x, params, lam


@pytest.mark.parametrize("flags,lanes", [(0, 1), (kcs.KCS_PLAN_GRAPH, 1), (kcs.KCS_PLAN_GRAPH, 2)])
def test_served_results_equal_alone(flags, lanes):
    reqs = small_stream()
    ex = serve.GpuExecutor(DEV, flags, n_lanes=lanes)
    comp, results, makespan, ticks = serve.serve(reqs, 1 << 40, ex, keep_results=True,
                                                 lane_of=lambda r: r.rid % lanes)
    ex.close()
    assert sorted(c.rid for c in comp) == list(range(len(reqs)))
    assert ticks < sum(r.n_sweeps for r in reqs)  # studies shared ticks
    for r in reqs:
        ref = alone(r)
        errs = [rel_l2(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(results[r.rid], ref)]
        print(f"request {r.rid} ({r.g.nx}x{r.g.ny}x{r.g.nz}, {r.n_sweeps} sweeps): mix vs alone {errs}")
        assert max(errs) <= 1e-5


def test_served_study_matches_oracle():
    """Two served studies of the mix (a 64x64 slice and a 40x40x3 stack) against the FP64 oracle's
    schedules: the served result equals, bit for bit, the study's schedule stepped one MAP-LM
    iteration at a time, whose decisions are compared with the oracle's iteration by iteration
    (image and decision-consistent maps within 1e-3; see test_gpu_schedule.py)."""
    reqs = small_stream()
    ex = serve.GpuExecutor(DEV, kcs.KCS_PLAN_GRAPH, n_lanes=2)
    comp, results, _, _ = serve.serve(reqs, 1 << 40, ex, keep_results=True, lane_of=lambda r: r.rid % 2)
    ex.close()
    assert len(comp) == len(reqs)
    for rid in (0, 2):
        r = reqs[rid]
        st = oracle.make_study(r.cfg)
        run, lams, xs, _ = run_gpu(st, r.n_sweeps, st.lm.eta, lockstep=False)
        for a, b in zip(results[rid], (run.x, run.params, run.lam)):
            assert torch.equal(a, b)
        ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, r.n_sweeps, st.lm.eta, lams, xs)
        check_independent(f"served {st.cfg.name}, {r.n_sweeps} sweeps,", st.lm.eta, st, host(run.x),
                          host(run.params), ox, op, first, margin, bound, inherited, max_diverged=0.02)


def test_served_under_tight_budget():
    """A budget that holds only two of the studies at a time: they queue, and still match."""
    reqs = small_stream()
    sizes = sorted(r.footprint() for r in reqs)
    budget = sizes[-1] + sizes[-2]
    ex = serve.GpuExecutor(DEV, n_lanes=2)
    comp, results, _, _ = serve.serve(reqs, budget, ex, keep_results=True, lane_of=lambda r: r.rid % 2)
    ex.close()
    assert len(comp) == len(reqs)
    for r in reqs[:3]:
        ref = alone(r)
        assert max(rel_l2(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(results[r.rid], ref)) <= 1e-5
