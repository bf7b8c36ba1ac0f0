"""GPU: the multiplicative correction sinogram (attenuation x detector efficiency, system matrix
diag(mu) P) through the C ABI against the FP64 oracle: projection, back projection with
sensitivity and adjointness, the OSL update, a short ICM schedule, and a plan."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from kcs_testutil import default_frames, geometry_pair, kcs_objects, make_image, rel_l2

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"
M = 24

GEOMS = {
    "disk64": (64, 64, 1, 4.0, 60, 64, 4.0, 0.0, 4),
    "ragged": (37, 29, 3, 2.3, 50, 45, 1.9, 0.05, 7),
    "wide_bins": (40, 44, 2, 2.0, 33, 23, 3.7, 0.0, 3),
    "brain344_1plane": (344, 344, 1, 2.09, 252, 344, 2.09, 0.0, 21),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def kframes(fr):
    return kcs.Frames(fr.t0, fr.t1, fr.E, fr.r)


def corrected(kg, mult):
    return dataclasses.replace(kg, mult=dev(mult))


def radius(nx, h):
    """A head-sized water cylinder (at most 100 mm radius, inside the field of view)."""
    return min(0.4 * nx * h, 100.0)


@pytest.mark.parametrize("name", list(GEOMS))
def test_project_with_correction(name):
    nx, ny, nz, h, na, nb, du, a0, Q = GEOMS[name]
    og, kg = geometry_pair(nx, ny, nz, h, na, nb, du, a0)
    mult = inputs.correction_sinogram(nz, na, nb, du, radius(nx, h))
    kg = corrected(kg, mult)
    fr = default_frames()
    x = make_image(nz, ny, nx, M, seed=1)
    for q in sorted({0, Q // 2, Q - 1}):
        ref = oracle.expected_counts(og, fr, x, q, Q, mult.astype(np.float64))
        out = torch.empty((nz, kg.subset_size(q, Q), nb, M), device=DEV)
        kcs.kcs_project(kg, kframes(fr), dev(x), q, Q, out)
        torch.cuda.synchronize()
        err = rel_l2(out.cpu().numpy(), ref)
        print(f"{name} q={q}: corrected project relL2 {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_backproject_with_correction(name):
    nx, ny, nz, h, na, nb, du, a0, Q = GEOMS[name]
    og, kg = geometry_pair(nx, ny, nz, h, na, nb, du, a0)
    mult = inputs.correction_sinogram(nz, na, nb, du, radius(nx, h), seed=22)
    kg = corrected(kg, mult)
    fr = default_frames()
    rng = np.random.default_rng(2)
    x = make_image(nz, ny, nx, M, seed=3)
    for q in sorted({0, Q // 2, Q - 1}):
        A = kg.subset_size(q, Q)
        mu = oracle.subset_mult(og, mult.astype(np.float64), q, Q)
        y = rng.random((nz, A, nb, M)).astype(np.float32).astype(np.float64)
        ref = fr.E * oracle.back(og, mu * y, q, Q)
        ref_sens = oracle.back(og, np.ascontiguousarray(mu), q, Q)[..., 0]
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
        print(f"{name} q={q}: corrected back {eb:.2e} sens {es:.2e} adjoint {adj:.2e}")
        assert eb < 1e-5 and es < 1e-5 and adj < 1e-5


def corrected_study(seed=31):
    """The 64x64 study with its sinogram regenerated through diag(mu) P (seeded Poisson counts)."""
    st = oracle.make_study(inputs.disk64())
    g = st.geom
    mult = inputs.correction_sinogram(g.nz, g.n_ang, g.n_bin, g.du, radius(g.nx, g.h)).astype(np.float64)
    ybar = oracle.expected_counts(g, st.frames, st.truth_x, 0, 1, mult)
    sino = inputs.poisson_counts(ybar, seed).astype(np.float64)
    return st, mult, sino


@pytest.mark.parametrize("kp", [False, True])
def test_osl_update_with_correction(kp):
    st, mult, sino = corrected_study()
    g, f, k, p, _ = kcs_objects(st)
    g = corrected(g, mult)
    rng = np.random.default_rng(5)
    x0 = (st.truth_x * (1 + 0.2 * rng.standard_normal(st.truth_x.shape)) + 0.05).clip(0.01)
    x0 = x0.astype(np.float32).astype(np.float64)
    maps = np.stack([np.full((1, 64, 64), v) for v in (0.09, 0.11, 0.05)])
    maps[:, st.mask] = st.truth_params[:, st.mask]
    maps = maps.astype(np.float32).astype(np.float64)
    pk = dataclasses.replace(p, kp_on=kp)
    work = kcs.alloc_workspace(g, M, 4, DEV)
    xd, sd = dev(x0), dev(sino)
    ox = x0.copy()
    for q in range(4):
        kcs.kcs_osl_update(g, f, k, pk, sd, dev(maps), q, 4, xd, work)
        ox = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, sino, maps, ox, q, 4, kp, mult)
        torch.cuda.synchronize()
        err = rel_l2(xd.cpu().numpy(), ox)
        print(f"corrected osl kp={kp} q={q}: relL2 {err:.2e}")
        assert err < 1e-5


def test_icm_schedule_with_correction():
    """4 sweeps of the 64x64 study with attenuation and efficiencies: the image to the
    whole-schedule tolerance over all voxels and the maps over the active voxels whose
    accept/reject path agreed with the oracle's in every sweep."""
    st, mult, sino = corrected_study()
    cfg = st.cfg
    g, f, k, p, lm = kcs_objects(st)
    g = corrected(g, mult)
    sd = dev(sino)
    x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lamd = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, M, cfg.Q, DEV)
    kcs.kcs_init_state(g, f, sd, inputs.XI0, x, params, lamd, work)
    ox, op, ol = oracle.initial_state(st.geom, st.frames, sino)
    diverged = np.zeros(ol.shape, dtype=bool)
    for s in range(4):
        kcs.kcs_icm_sweep(g, f, k, p, lm, sd, cfg.Q, s, x, params, lamd, work)
        ox, op, ol = oracle.icm_sweep(st.geom, st.frames, st.kin, st.prior, st.lm, sino, ox, op, ol, cfg.Q, s, mult)
        diverged |= np.abs(lamd.cpu().numpy() / ol - 1.0) > 1e-3
    gx, gp = x.cpu().numpy(), params.cpu().numpy()
    act = (ox * (st.frames.t1 - st.frames.t0)).sum(axis=-1)
    keep = (act >= 0.1 * act.max()) & ~diverged
    ex = rel_l2(gx, ox)
    maps = [rel_l2(gp[i][keep], op[i][keep]) for i in range(3)]
    print(f"corrected 64x64, 4 sweeps: image {ex:.2e}, maps {maps} ({int(diverged.sum())} voxels on another path)")
    assert ex < 1e-3 and max(maps) < 1e-3
    assert diverged[act >= 0.1 * act.max()].mean() < 0.02


def test_plan_with_correction_matches_plain_calls():
    st, mult, sino = corrected_study()
    cfg = st.cfg
    g, f, k, p, lm = kcs_objects(st)
    g = corrected(g, mult)
    sd = dev(sino)
    states = []
    for _ in range(2):
        x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
        params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
        lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
        work = kcs.alloc_workspace(g, M, cfg.Q, DEV)
        kcs.kcs_init_state(g, f, sd, inputs.XI0, x, params, lam, work)
        states.append((x, params, lam, work))
    x, params, lam, work = states[0]
    for s in range(2):
        kcs.kcs_icm_sweep(g, f, k, p, lm, sd, cfg.Q, s, x, params, lam, work)
    x2, params2, lam2, work2 = states[1]
    plan = kcs.kcs_plan_create([kcs.Study(g, f, k, p, lm, cfg.Q, 0, 2, sd, x2, params2, lam2, work2)],
                               kcs.KCS_PLAN_GRAPH)
    kcs.kcs_plan_run(plan)
    torch.cuda.synchronize()
    kcs.kcs_plan_destroy(plan)
    for a, b in ((x, x2), (params, params2), (lam, lam2)):
        err = rel_l2(b.cpu().numpy(), a.cpu().numpy())
        assert err < 1e-6, err
