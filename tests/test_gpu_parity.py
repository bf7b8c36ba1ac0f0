"""GPU parity: every entry point of the HIP library against the FP64 oracle on the same
seeded inputs (relative L2 tolerances: 1e-5 for one projection / back projection / update,
1e-3 for images and kinetic maps after the whole ICM schedule)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from kcs_testutil import (decision_bound, default_frames, geometry_pair, kcs_objects, make_image,
                          oracle_fit_history, path_consistent, rel_l2, same_fit_path)

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402
from gpu_schedule_util import gpu_fit_history  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"

KIN = oracle.Kinetics(**inputs.FENG, vb=inputs.VB)
T0, T1 = inputs.frame_times()
M = len(T0)

GEOMS = {
    "disk64": (64, 64, 1, 4.0, 60, 64, 4.0, 0.0, 4),
    "ragged": (37, 29, 3, 2.3, 50, 45, 1.9, 0.05, 7),  # uneven subsets, bins narrower than pixels
    "wide_bins": (40, 44, 2, 2.0, 33, 23, 3.7, 0.0, 3),  # bins wider than pixels: > 2 bins per voxel
    "brain128_2planes": (128, 128, 2, 2.5, 168, 128, 2.5, 0.0, 6),
    "brain344_1plane": (344, 344, 1, 2.09, 252, 344, 2.09, 0.0, 21),
}


def kframes(fr):
    return kcs.Frames(fr.t0, fr.t1, fr.E, fr.r)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def subsets_to_test(Q):
    return sorted({0, Q // 2, Q - 1})


@pytest.mark.parametrize("name", list(GEOMS))
def test_project_parity(name):
    nx, ny, nz, h, na, nb, du, a0, Q = GEOMS[name]
    og, kg = geometry_pair(nx, ny, nz, h, na, nb, du, a0)
    fr = default_frames()
    x = make_image(nz, ny, nx, M, seed=1)
    xd = dev(x)
    for q in subsets_to_test(Q):
        ref = oracle.expected_counts(og, fr, x, q, Q)
        out = torch.empty((nz, kg.subset_size(q, Q), nb, M), device=DEV)
        kcs.kcs_project(kg, kframes(fr), xd, q, Q, out)
        torch.cuda.synchronize()
        err = rel_l2(out.cpu().numpy(), ref)
        print(f"{name} q={q}: project relL2 {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_backproject_parity_and_adjointness(name):
    nx, ny, nz, h, na, nb, du, a0, Q = GEOMS[name]
    og, kg = geometry_pair(nx, ny, nz, h, na, nb, du, a0)
    fr = default_frames()
    rng = np.random.default_rng(2)
    x = make_image(nz, ny, nx, M, seed=3)
    for q in subsets_to_test(Q):
        A = kg.subset_size(q, Q)
        y = rng.random((nz, A, nb, M)).astype(np.float32).astype(np.float64)
        ref = fr.E * oracle.back(og, y, q, Q)
        ref_sens = np.broadcast_to(oracle.subset_sensitivity(og, q, Q), (nz, ny, nx))
        b = torch.empty((nz, ny, nx, M), device=DEV)
        sens = torch.empty((nz, ny, nx), device=DEV)
        kcs.kcs_backproject(kg, kframes(fr), dev(y), q, Q, b, sens)
        ax = torch.empty((nz, A, nb, M), device=DEV)
        kcs.kcs_project(kg, kframes(fr), dev(x), q, Q, ax)
        torch.cuda.synchronize()
        eb, es = rel_l2(b.cpu().numpy(), ref), rel_l2(sens.cpu().numpy(), ref_sens)
        lhs = np.sum((ax.cpu().numpy().astype(np.float64) - fr.r) * y)
        rhs = np.sum(x * b.cpu().numpy().astype(np.float64))
        adj = abs(lhs - rhs) / abs(lhs)
        print(f"{name} q={q}: back {eb:.2e} sens {es:.2e} adjoint {adj:.2e}")
        assert eb < 1e-5 and es < 1e-5 and adj < 1e-5


def model_params():
    P = [inputs.WHITE, inputs.GRAY, inputs.HOT, (0.75, 0.35, 0.031), (0.51, 0.27, 0.018),
         (0.2, 1e-4, 0.0), (0.05, 2.0, 1.0), (1.0, 1e-4, 1e-3), (2.0, 0.0, 1e-4)]
    for lam in (KIN.l1, KIN.l2, KIN.l3):  # k2 + k3 at and around -lambda_i (removable singularity)
        for eps in (0.0, 1e-7, -1e-7, 1e-4, -1e-4, 3e-3, -3e-3, 0.02, -0.02):
            a = -lam + eps
            if a > 0:
                P.append((0.1, 0.6 * a, 0.4 * a))
    rng = np.random.default_rng(4)
    lo, hi = np.array(inputs.LM_LO), np.array(inputs.LM_HI)
    P += list(rng.uniform(lo, [1.0, 1.0, 0.5], (400, 3)))
    P += list(rng.uniform([0.01, 0.01, 0.0], [0.2, 0.4, 0.2], (400, 3)))
    return np.array(P, dtype=np.float32).astype(np.float64)


def test_model_tac_parity():
    P = model_params()
    n = len(P)
    fr = default_frames()
    kk = kcs.Kinetics(KIN.A1, KIN.A2, KIN.A3, KIN.l1, KIN.l2, KIN.l3, KIN.vb)
    F = torch.empty((n, M), device=DEV)
    J = torch.empty((n, M, 3), device=DEV)
    work = kcs.alloc_workspace(None, M, 0, DEV)
    kcs.kcs_model_tac(kframes(fr), kk, dev(P.T.copy()), F, J, work)
    torch.cuda.synchronize()
    Fo, Jo = oracle.model_tac(P, T0, T1, KIN, jacobian=True)
    Fg, Jg = F.cpu().numpy().astype(np.float64), J.cpu().numpy().astype(np.float64)
    fe = np.linalg.norm(Fg - Fo, axis=1) / np.linalg.norm(Fo, axis=1)
    je = np.linalg.norm(Jg - Jo, axis=1) / np.maximum(np.linalg.norm(Jo, axis=1), 1e-30)
    worst = np.argmax(fe)
    print(f"model: max F relL2 {fe.max():.2e} at {P[worst]}, median {np.median(fe):.2e}; "
          f"max J relL2 per column {je.max(axis=0)}")
    # FP32 limit: int C_T = K1 (P2 - k2 J) cancels when k3 << k2 (washout), ~40 ulp at k2 = 2
    inbox = (P[:, 1] <= inputs.LM_HI[1]) & (P[:, 2] <= inputs.LM_HI[2])
    assert fe[inbox].max() < 5e-6 and fe.max() < 2e-5
    assert np.all(je[inbox].max(axis=0) < 5e-5)


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 37, 29), (2, 128, 129)])
def test_ki_map_parity(shape):
    """K_i map against the oracle's net_influx on random maps in and beyond the box, with k2 = 0,
    k3 = 0 and k2 = k3 = 0 among them; sizes with a ragged last workgroup."""
    rng = np.random.default_rng(7)
    P = np.stack([rng.uniform(0.0, 1.0, shape), rng.uniform(0.0, 2.0, shape), rng.uniform(0.0, 1.0, shape)])
    flat = P.reshape(3, -1)
    if flat.shape[1] >= 3:
        flat[1, 0] = 0.0
        flat[2, 1] = 0.0
        flat[1:, 2] = 0.0
    P = flat.reshape(P.shape).astype(np.float32)
    ki = torch.empty(shape, device=DEV)
    kcs.kcs_ki_map(dev(P), ki)
    torch.cuda.synchronize()
    ref = oracle.net_influx(P.astype(np.float64))
    got = ki.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)
    print(f"K_i map {shape}: max rel err {err.max():.2e}")
    assert np.all(np.isfinite(got)) and err.max() < 1e-6


def disk64_study():
    return oracle.make_study(inputs.disk64())


def test_init_state_parity():
    st = disk64_study()
    g, f, *_ = kcs_objects(st)
    x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, M, 0, DEV)
    kcs.kcs_init_state(g, f, dev(st.sino), inputs.XI0, x, params, lam, work)
    torch.cuda.synchronize()
    ox, op, ol = oracle.initial_state(st.geom, st.frames, st.sino.astype(np.float64))
    assert rel_l2(x.cpu().numpy(), ox) < 1e-6
    assert rel_l2(params.cpu().numpy(), op) < 1e-7
    assert np.all(lam.cpu().numpy() == 0)


@pytest.mark.parametrize("kp", [False, True])
def test_osl_update_parity(kp):
    st = disk64_study()
    g, f, k, p, _ = kcs_objects(st)
    rng = np.random.default_rng(5)
    x0 = (st.truth_x * (1 + 0.2 * rng.standard_normal(st.truth_x.shape)) + 0.05).clip(0.01)
    x0 = x0.astype(np.float32).astype(np.float64)
    maps = np.stack([np.full((1, 64, 64), v) for v in (0.09, 0.11, 0.05)])
    maps[:, st.mask] = st.truth_params[:, st.mask]
    maps = maps.astype(np.float32).astype(np.float64)
    pk = kcs.Prior(p.beta_kp, p.eps_F, p.beta_h, p.delta, kp)
    work = kcs.alloc_workspace(g, M, 4, DEV)
    xd = dev(x0)
    sino = dev(st.sino)
    ox = x0.copy()
    for q in range(4):
        kcs.kcs_osl_update(g, f, k, pk, sino, dev(maps), q, 4, xd, work)
        ox = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, st.sino.astype(np.float64), maps, ox, q, 4, kp)
        torch.cuda.synchronize()
        err = rel_l2(xd.cpu().numpy(), ox)
        print(f"osl kp={kp} q={q}: relL2 {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("eta", [inputs.LM_ETA, 0.0])
def test_lm_fit_parity(eta):
    """A 5-iteration fit of the 64x64 slice from the initial maps, with the relative sufficient
    decrease (eta = 1e-3) and with the plain strict decrease (eta = 0), over the object voxels whose
    decisions agreed with the oracle's in every iteration."""
    st = disk64_study()
    st = dataclasses.replace(st, lm=dataclasses.replace(st.lm, eta=eta))
    g, f, k, p, lm = kcs_objects(st)
    rng = np.random.default_rng(6)
    x = st.truth_x * (1 + 0.05 * rng.standard_normal(st.truth_x.shape))
    x = x.astype(np.float32).astype(np.float64)
    params0 = np.stack([np.full((1, 64, 64), v) for v in inputs.XI0])
    lam0 = np.zeros((1, 64, 64))
    gp, gl, gh = gpu_fit_history(g, f, k, p, lm, x, params0, lam0)
    op, ol, oh = oracle_fit_history(st, st.prior, st.lm, x, params0, lam0)
    # an accept test within rounding of its threshold may go the other way (see the near-tie test)
    same = same_fit_path(gh, oh)
    mask = st.mask
    keep = mask & same
    for i in range(3):
        e = rel_l2(gp[i][keep], op[i][keep])
        print(f"eta={eta} lm param {i}: relL2 over object voxels with the oracle's LM path {e:.2e} "
              f"(all object voxels {rel_l2(gp[i][mask], op[i][mask]):.2e}; other path {int((mask & ~same).sum())})")
        assert e < 1e-4
    # under the strict decrease a voxel at its optimum ties every iteration (dPhi = 0 to FP32
    # resolution), so many voxels take the other branch somewhere in the fit; their decisions are
    # checked one by one against the FP32 bound in test_gpu_schedule.py
    if eta > 0:
        assert same[mask].mean() > 0.99


def test_lm_fit_parity_3x3x3_neighbourhood():
    """The fit with the 3x3x3 Huber neighbourhood (planes 0.97 pixel sides apart) on a 3-plane
    128x128 stack against the oracle, over the object voxels whose decisions and whose
    neighbours' decisions agreed with the oracle's in every iteration."""
    cfg = inputs.scaled(inputs.batch_configs()[3], nz=3, counts=4e5 * 3)
    st = oracle.make_study(cfg)
    prior = dataclasses.replace(st.prior, plane_ratio=0.97)
    g, f, k, p, lm = kcs_objects(st)
    p = dataclasses.replace(p, plane_ratio=0.97)
    rng = np.random.default_rng(8)
    x = st.truth_x * (1 + 0.05 * rng.standard_normal(st.truth_x.shape))
    x = x.astype(np.float32).astype(np.float64)
    shp = x.shape[:3]
    params0 = np.stack([np.full(shp, v) for v in inputs.XI0])
    lam0 = np.zeros(shp)
    gp, gl, gh = gpu_fit_history(g, f, k, p, lm, x, params0, lam0)
    op, ol, oh = oracle_fit_history(st, prior, st.lm, x, params0, lam0)
    same = same_fit_path(gh, oh)
    # a voxel on another path moves its 26 neighbours' Huber gradients: those are left out too
    keep = st.mask & path_consistent(same, nbr3d=True)
    for i in range(3):
        e = rel_l2(gp[i][keep], op[i][keep])
        print(f"3x3x3 lm param {i}: relL2 {e:.2e} over object voxels on the oracle's path with their "
              f"neighbours ({int((st.mask & ~same).sum())} of {int(st.mask.sum())} on another; "
              f"{int((st.mask & same & ~keep).sum())} beside one)")
        assert e < 1e-4
    assert same[st.mask].mean() > 0.99


@pytest.mark.parametrize("tile", ["0", "16", "32", "64"])
def test_osl_update_projector_variants(tile, monkeypatch):
    """The OSL update with each forward-projector variant (ray-driven, LDS tiles of 16, 32 or 64
    pixels with partial sums; 32 and 64 stage half and a quarter of the frames per workgroup) on a
    geometry with ragged edge tiles and uneven subsets."""
    monkeypatch.setenv("KCS_PROJ_TILE", tile)
    nx, ny, nz, h, na, nb, du, Q = 150, 130, 2, 2.0, 100, 160, 1.8, 7
    og, kg = geometry_pair(nx, ny, nz, h, na, nb, du, 0.02)
    fr = default_frames(seed=3)
    rng = np.random.default_rng(7)
    x0 = make_image(nz, ny, nx, M, seed=8)
    sino = rng.poisson(fr.E * oracle.forward(og, x0) + fr.r).astype(np.float32).astype(np.float64)
    maps = np.stack([np.full((nz, ny, nx), v) for v in inputs.GRAY])
    prior = oracle.Prior(beta_kp=0.1, eps_F=0.01, beta_h=0.1, delta=(1e-3,) * 3, kp_on=False)
    kp = kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3, False)
    kk = kcs.Kinetics(KIN.A1, KIN.A2, KIN.A3, KIN.l1, KIN.l2, KIN.l3, KIN.vb)
    work = kcs.alloc_workspace(kg, M, Q, DEV)
    xd = dev(x0)
    ox = x0.copy()
    for q in range(Q):
        kcs.kcs_osl_update(kg, kframes(fr), kk, kp, dev(sino), dev(maps), q, Q, xd, work)
        ox = oracle.osl_update(og, fr, KIN, prior, sino, maps, ox, q, Q, False)
    torch.cuda.synchronize()
    err = rel_l2(xd.cpu().numpy(), ox)
    print(f"projector tile {tile}: OSL pass relL2 {err:.2e}")
    assert err < 1e-5


# ---------------------------------------------------------------------------------------------
# MAP-LM accept decisions.  The accept test compares the change of the voxel objective with a
# fraction eta of it; where the two lie within the FP32 evaluation error of each other either
# branch is a result of the method.  Every decision that differs from the oracle's on the same
# state must be such a near-tie (whole schedules: test_gpu_schedule.py).

def low_count_plane_state(n_iter_before=3):
    """A mid-fit MAP-LM state on a low-count 128x128 plane (the batch recipe's counts per plane):
    the oracle's image after one OS-EM pass and its maps and lambda after `n_iter_before` LM
    iterations, all rounded to FP32."""
    cfg = inputs.scaled(inputs.batch_configs()[3], nz=1, counts=4e5)
    st = oracle.make_study(cfg)
    sino = st.sino.astype(np.float64)
    x, p0, lam0 = oracle.initial_state(st.geom, st.frames, sino)
    for q in range(cfg.Q):
        x = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, sino, p0, x, q, cfg.Q, False)
    x = x.astype(np.float32).astype(np.float64)
    opt = oracle.LMOptions(n_iter_before, st.lm.tau, st.lm.lam_min, st.lm.lam_max, st.lm.lo, st.lm.hi, st.lm.eta)
    p, lam = oracle.lm_fit(st.frames, st.kin, st.prior, opt, x, p0, np.zeros_like(lam0))
    return st, x, p.astype(np.float32).astype(np.float64), lam.astype(np.float32).astype(np.float64)


def test_lm_decisions_differ_only_at_near_ties():
    st, x, p, lam = low_count_plane_state()
    g, f, k, pr, lm = kcs_objects(st)
    one = kcs.LMOptions(1, lm.tau, lm.lam_min, lm.lam_max, lm.lo, lm.hi, lm.eta)
    work = kcs.alloc_workspace(g, M, 0, DEV)
    pd, ld = dev(p), dev(lam)
    kcs.kcs_lm_fit(g, f, k, pr, one, dev(x), pd, ld, work)
    torch.cuda.synchronize()
    opt1 = oracle.LMOptions(1, st.lm.tau, st.lm.lam_min, st.lm.lam_max, st.lm.lo, st.lm.hi, st.lm.eta)
    op, ol, phi0, phi1 = oracle.lm_iteration(st.frames, st.kin, st.prior, opt1, x, p, lam, with_objective=True)
    g_acc = ld.cpu().numpy() < lam
    o_acc = ol < lam
    differ = g_acc != o_acc
    eta = st.lm.eta
    ratio = np.abs(phi1 - phi0 + eta * phi0) / decision_bound(x, phi0, phi1)
    print(f"one LM iteration on {x.shape[1]}x{x.shape[2]}: {int(differ.sum())} of {differ.size} decisions differ; "
          f"their oracle margins in units of the FP32 bound {np.sort(ratio[differ])[:10]}")
    assert differ.mean() < 1e-3
    assert np.all(ratio[differ] <= 1.0)
    gp = pd.cpu().numpy()
    same = ~differ
    for i in range(3):
        e = rel_l2(gp[i][same], op[i][same])
        print(f"  map {i} over voxels with the same decision: relL2 {e:.2e}")
        assert e < 1e-4
