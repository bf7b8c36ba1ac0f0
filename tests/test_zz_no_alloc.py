"""kcs_icm_sweep_noalloc (the library's static per-GPU scratch as workspace) against
kcs_icm_sweep with a caller workspace: the same kernels on the same inputs, so the results must be
identical.  Two calls in a row, the second on a smaller study, so that the second one runs on
scratch left over from the first."""
import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from kcs_testutil import kcs_objects

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"
M = 24


def initial(st, g, f, sino):
    x = torch.empty((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.empty((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.empty((g.nz, g.ny, g.nx), device=DEV)
    work = kcs.alloc_workspace(g, M, 0, DEV)
    kcs.kcs_init_state(g, f, sino, inputs.XI0, x, params, lam, work)
    return x, params, lam


def sweeps(st, n_sweeps, noalloc):
    g, f, k, p, lm = kcs_objects(st)
    sino = torch.from_numpy(st.sino).to(DEV)
    x, params, lam = initial(st, g, f, sino)
    work = None if noalloc else kcs.alloc_workspace(g, M, st.cfg.Q, DEV)
    for s in range(n_sweeps):
        if noalloc:
            kcs.kcs_icm_sweep_noalloc(g, f, k, p, lm, sino, st.cfg.Q, s, x, params, lam)
        else:
            kcs.kcs_icm_sweep(g, f, k, p, lm, sino, st.cfg.Q, s, x, params, lam, work)
    torch.cuda.synchronize()
    return x.cpu().numpy(), params.cpu().numpy(), lam.cpu().numpy()


def test_noalloc_sweep_equals_workspace_sweep():
    big = oracle.make_study(inputs.scaled(inputs.batch_configs()[3], nz=3, counts=4e5 * 3))  # 128x128x3, Q = 6
    small = oracle.make_study(inputs.disk64())  # 64x64x1, Q = 4
    g_big = kcs_objects(big)[0]
    need = kcs.kcs_workspace_bytes(g_big, M, big.cfg.Q)
    assert kcs.kcs_workspace_bytes(kcs_objects(small)[0], M, small.cfg.Q) < need <= 256 << 20
    for st, n in ((big, 3), (small, 2)):
        ref = sweeps(st, n, noalloc=False)
        got = sweeps(st, n, noalloc=True)
        print(f"{st.cfg.name}: {n} sweeps through the static scratch")
        for a, b, name in zip(got, ref, ("image", "maps", "lambda")):
            assert np.array_equal(a, b), name


def test_noalloc_rejects_a_study_beyond_the_scratch():
    cfg = inputs.scaled(inputs.brain128(), nz=60)
    g = kcs.Geometry.from_config(cfg)
    assert kcs.kcs_workspace_bytes(g, M, cfg.Q) > 256 << 20
    st_small = oracle.make_study(inputs.disk64())
    _, f, k, p, lm = kcs_objects(st_small)
    sino = torch.zeros((g.nz, g.n_ang, g.n_bin, M), device=DEV)
    x = torch.ones((g.nz, g.ny, g.nx, M), device=DEV)
    params = torch.ones((3, g.nz, g.ny, g.nx), device=DEV)
    lam = torch.zeros((g.nz, g.ny, g.nx), device=DEV)
    with pytest.raises(kcs.KcsError) as e:
        kcs.kcs_icm_sweep_noalloc(g, f, k, p, lm, sino, cfg.Q, 0, x, params, lam)
    assert e.value.code == kcs.KCS_EWORKSPACE and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(x == 1.0)  # nothing launched
