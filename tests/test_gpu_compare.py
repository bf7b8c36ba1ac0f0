"""GPU: the method comparison (INDIRECT, DIRECT, KCS DIRECT) on the ring phantom.  The method
switches are checked against the FP64 oracle run with the same prior settings, and the batched
runner of many noise realizations is exercised end to end."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import compare, inputs
from kcs_testutil import kcs_objects, rel_l2

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("method", compare.METHODS)
def test_method_settings_match_oracle(method):
    """3 sweeps of the 64x64 ring study under each method's prior settings against the oracle
    run with the same settings (image over all voxels, maps over active voxels on the oracle's
    accept/reject path)."""
    st = oracle.make_study(inputs.rings_config(64, nz=1, counts_per_plane=2e6))
    g, f, k, p, lm = kcs_objects(st)
    pm = compare.method_prior(p, method, st.prior.beta_h)
    po = dataclasses.replace(st.prior, kp_on=pm.kp_on, beta_h=pm.beta_h)
    Q = st.cfg.Q
    sd = dev(st.sino)
    x = torch.empty((g.nz, g.ny, g.nx, f.M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, f.M, Q, DEV)
    kcs.kcs_init_state(g, f, sd, inputs.XI0, x, params, lam, work)
    sino = st.sino.astype(np.float64)
    ox, op, ol = oracle.initial_state(st.geom, st.frames, sino)
    diverged = np.zeros(ol.shape, dtype=bool)
    for s in range(3):
        kcs.kcs_icm_sweep(g, f, k, pm, lm, sd, Q, s, x, params, lam, work)
        ox, op, ol = oracle.icm_sweep(st.geom, st.frames, st.kin, po, st.lm, sino, ox, op, ol, Q, s)
        diverged |= np.abs(lam.cpu().numpy() / ol - 1.0) > 1e-3
    gx, gp = x.cpu().numpy(), params.cpu().numpy()
    act = (ox * (st.frames.t1 - st.frames.t0)).sum(axis=-1)
    active = act >= 0.1 * act.max()
    keep = active & ~diverged
    ex = rel_l2(gx, ox)
    maps = [rel_l2(gp[i][keep], op[i][keep]) for i in range(3)]
    print(f"{method}: image {ex:.2e}, maps {['%.2e' % e for e in maps]}, other path {int((active & diverged).sum())}")
    assert ex < 1e-3 and max(maps) < 1e-3 and diverged[active].mean() < 0.02


def test_batched_realizations_runner():
    cfg = inputs.rings_config(64, nz=2, counts_per_plane=1e6)
    g, f, kin, prior, lm, ybar, maps, labels = compare.synthesize_truth(cfg, DEV)
    sinos = [compare.realization(ybar, 100 + r) for r in range(3)]
    assert not torch.equal(sinos[0], sinos[1])
    res = compare.run_method(g, f, kin, compare.method_prior(prior, "kcs", cfg.beta_h), lm, sinos, cfg.Q, 2, (1, 2),
                             DEV)
    assert sorted(res) == [1, 2] and res[2].shape == (3, 4, 2, 64, 64)
    # the K_i channel is the library's map of the fitted maps
    np.testing.assert_allclose(res[2][:, 3], compare.true_ki(np.moveaxis(res[2][:, :3], 1, 0)), rtol=1e-5, atol=1e-7)
    rows = compare.summarize(res, maps, labels)
    assert len(rows) == 2 * 3 * 2
    assert all(np.isfinite(r["bias_pct"]) and np.isfinite(r["std_pct"]) and r["std_pct"] > 0 for r in rows)
