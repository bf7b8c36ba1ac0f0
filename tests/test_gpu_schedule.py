"""Whole ICM schedules (Sec. II-D: OS-MAP-OSL-KP passes alternating with MAP-LM fits, lambda
restarted every sweep) on the GPU against the FP64 oracle, on the 64x64 slice and on planes cut
from the two 3D studies with the counts they carry there (central plane and a lesion plane).

Two comparisons per schedule:
  * lockstep: before every GPU MAP-LM iteration the oracle takes the GPU's own state (image, maps,
    damping) and makes the same iteration in FP64; every decision that differs must be one the
    FP32 evaluation cannot resolve (oracle margin |dPhi + eta Phi| within the evaluation bound of
    kcs_testutil.decision_bound), and the maps of the agreeing voxels must match;
  * independent: the oracle runs the schedule from its own initial state; the image must match
    over all voxels, the maps over the active voxels whose decisions agreed in every iteration, and
    each other voxel's first differing decision must be within the bound (widened by the states'
    image difference).  The maps over all active voxels are reported.

Both acceptance readings run: eta = 1e-3 (relative sufficient decrease, the default) and eta = 0
(the plain strict decrease), under which a voxel at its optimum makes a tie every iteration.

The GPU runs the schedule through kcs_osl_update and single-iteration kcs_lm_fit calls (so every
decision is seen) and through kcs_icm_sweep at the full size of the study (the sampled planes
repeated to the study's plane count, the launch configuration the benchmark times); the two
must give the same planes bit for bit."""
import concurrent.futures as cf
import dataclasses
import multiprocessing as mp

import numpy as np
import pytest

import oracle
from paper_1803_10045_amd import inputs
from gpu_schedule_util import assert_same_as_icm_sweeps, check_independent, check_lockstep, host, run_gpu
from kcs_testutil import oracle_schedule_vs_gpu, oracle_schedule_worker

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"

PLANES = {"brain128": (23, 34), "brain344": (63, 92)}  # central plane, plane with the most lesion voxels


@pytest.mark.parametrize("eta", [inputs.LM_ETA, 0.0])
def test_schedule_disk64(eta):
    """The 64x64 slice, 10 sweeps of 4 subsets and 5 LM iterations."""
    st = oracle.make_study(inputs.disk64())
    run, lams, xs, stats = run_gpu(st, st.cfg.n_sweeps, eta, lockstep=True)
    check_lockstep("disk64", eta, stats, max_frac=1e-4 if eta > 0 else 0.2)
    assert_same_as_icm_sweeps(run, st.cfg.n_sweeps)
    ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, st.cfg.n_sweeps, eta, lams, xs)
    check_independent("disk64", eta, st, host(run.x), host(run.params), ox, op, first, margin, bound,
                      inherited, max_diverged=2e-3 if eta > 0 else 1.0)


@pytest.mark.parametrize("eta", [inputs.LM_ETA, 0.0])
def test_schedule_brain128_planes(eta):
    """Planes 23 (centre) and 34 (lesions) of the 128x128x47 study, 20 sweeps of 6 subsets; the
    full-size run repeats them to 47 planes."""
    cfg = inputs.brain128()
    st = oracle.make_plane_study(cfg, PLANES["brain128"])
    run, lams, xs, stats = run_gpu(st, cfg.n_sweeps, eta, lockstep=True)
    check_lockstep("brain128 planes", eta, stats, max_frac=1e-4 if eta > 0 else 0.1)
    if eta == 0.0:
        return  # the lockstep is the check of the strict reading; the schedule is compared at eta > 0
    fx, fp, fl = run.full_size_sweeps(cfg.nz, cfg.n_sweeps)
    gx, gp, gl = run.x.cpu().numpy(), run.params.cpu().numpy(), run.lam.cpu().numpy()
    for z in range(cfg.nz):
        w = z % st.geom.nz
        assert np.array_equal(fx[z], gx[w]) and np.array_equal(fp[:, z], gp[:, w]) and np.array_equal(fl[z], gl[w]), z
    ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, cfg.n_sweeps, eta, lams, xs)
    check_independent("brain128 planes", eta, st, gx, gp, ox, op, first, margin, bound, inherited,
                      max_diverged=0.03)


# At the clinical-scale planes the schedule's image ends within 3e-3 of the oracle's, not 1e-3.
# The early 10-30 s frames carry almost no counts per plane there; their OS-EM images are a few
# isolated spikes, so a ray's line integral can be dominated by a corner chord of a few microns
# through one spike.  The projectors place each ray relative to the tile or voxel tile it crosses
# (FP64 reference, FP32 offsets of the tile's size), which keeps such chords to ~1e-6 pixel, but a
# few 1e-5 remain on each OSL pass (checked in lockstep below).  About 2 % of the voxels' fits
# then take another accept/reject path, and the kinetics-derived prior carries their maps back
# into the image.  Lockstep parity of every OSL pass and MAP-LM iteration holds as at the other sizes.
# The margins of the first differing decisions of the independent runs are reported, not
# asserted, at this size: besides the image, the two states differ there by the rounding of the
# maps along the shared path (accepted FP32 steps), which the bound does not cover; the lockstep
# check above is what pins each decision of the kernel.
BRAIN344_IMAGE_TOL = 3e-3
BRAIN344_OSL_TOL = 5e-5


def test_schedule_brain344_planes():
    """Planes 63 (centre) and 92 (lesions) of the 344x344x127 study, its 10 sweeps of 21 subsets;
    the full-size run repeats them to 127 planes.  Lockstep of the OSL passes of the first two
    sweeps; the oracle's own schedule runs one plane per process."""
    cfg = inputs.brain344()
    eta = inputs.LM_ETA
    st = oracle.make_plane_study(cfg, PLANES["brain344"])
    run, lams, xs, stats = run_gpu(st, cfg.n_sweeps, eta, lockstep=True, osl_lockstep_sweeps=2)
    check_lockstep("brain344 planes", eta, stats, max_frac=1e-4, osl_tol=BRAIN344_OSL_TOL)
    fx, fp, fl = run.full_size_sweeps(cfg.nz, cfg.n_sweeps)
    gx, gp, gl = run.x.cpu().numpy(), run.params.cpu().numpy(), run.lam.cpu().numpy()
    for z in range(cfg.nz):
        w = z % st.geom.nz
        assert np.array_equal(fx[z], gx[w]) and np.array_equal(fp[:, z], gp[:, w]) and np.array_equal(fl[z], gl[w]), z
    del fx, fp, fl
    # the oracle's initial state of the two-plane study, then one process per plane
    ix, ip, il = oracle.initial_state(st.geom, st.frames, st.sino.astype(np.float64))
    jobs = []
    for w in range(st.geom.nz):
        sub = dataclasses.replace(st, cfg=inputs.scaled(st.cfg, nz=1), geom=dataclasses.replace(st.geom, nz=1),
                                  sino=st.sino[w:w + 1], truth_params=st.truth_params[:, w:w + 1],
                                  truth_x=st.truth_x[w:w + 1], mask=st.mask[w:w + 1])
        state = (ix[w:w + 1].copy(), ip[:, w:w + 1].copy(), il[w:w + 1].copy())
        jobs.append((sub, cfg.n_sweeps, eta, lams[:, w:w + 1], xs[:, w:w + 1], state, 8))
    with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(oracle_schedule_worker, jobs))
    ox = np.concatenate([r[0] for r in res]).astype(np.float64)
    op = np.concatenate([r[1] for r in res], axis=1)
    first, margin, bound, inherited = (np.concatenate([r[k] for r in res]) for k in (3, 4, 5, 6))
    check_independent("brain344 planes", eta, st, gx.astype(np.float64), gp.astype(np.float64), ox, op, first,
                      margin, bound, inherited, max_diverged=0.03, image_tol=BRAIN344_IMAGE_TOL,
                      margin_check=False)


def test_schedule_low_count_64x64x2():
    """Two 64x64 planes at 4e5 counts each (the batch recipe's counts per plane: noisier fits
    than the single slice, so more near-tie decisions), 10 sweeps of 6 subsets."""
    cfg = inputs.StudyConfig("low_count_64x64x2", 64, 64, 2, 4.0, 4.0, 60, 64, 4.0, 8e5, 0.1, Q=6, n_sweeps=10,
                             phantom="brain", n_lesions=3, seed=31)
    st = oracle.make_study(cfg)
    eta = inputs.LM_ETA
    run, lams, xs, stats = run_gpu(st, cfg.n_sweeps, eta, lockstep=True)
    check_lockstep("low-count 64x64x2", eta, stats, max_frac=1e-4)
    assert_same_as_icm_sweeps(run, cfg.n_sweeps)
    ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, cfg.n_sweeps, eta, lams, xs)
    check_independent("low-count 64x64x2", eta, st, host(run.x), host(run.params), ox, op, first, margin, bound,
                      inherited, max_diverged=0.02)
