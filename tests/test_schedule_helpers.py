"""Host logic of the GPU schedule tests, checked on the CPU: the decision bookkeeping finds no
divergence when the 'GPU' record is the oracle's own, and finds a planted one at its iteration;
the plane studies carry the whole study's calibration."""
import dataclasses

import numpy as np

import oracle
from paper_1803_10045_amd import inputs
from kcs_testutil import decision_bound, gpu_accepted, oracle_decisions, oracle_schedule_vs_gpu


def small_study():
    cfg = inputs.scaled(inputs.disk64(), nx=16, ny=16, n_bin=16, n_ang=12, pixel_mm=16.0, bin_mm=16.0, Q=3,
                        counts=2e5)
    return oracle.make_study(cfg)


def oracle_record(st, n_sweeps, eta):
    """The oracle schedule with its damping after every iteration and image after every sweep."""
    opt = dataclasses.replace(st.lm, eta=eta, n_iter=1)
    sino = st.sino.astype(np.float64)
    x, p, lam = oracle.initial_state(st.geom, st.frames, sino)
    lams, xs, accs = [], [], []
    for s in range(n_sweeps):
        kp = s > 0
        for q in range(st.cfg.Q):
            x = oracle.osl_update(st.geom, st.frames, st.kin, st.prior, sino, p, x, q, st.cfg.Q, kp)
        xs.append(x.copy())
        lam = np.zeros_like(lam)
        for it in range(st.lm.n_iter):
            p, lam, acc, *_ = oracle_decisions(st, opt, x, p, lam)
            lams.append(lam.copy())
            accs.append(acc)
    return np.stack(lams), np.stack(xs), np.stack(accs), x, p


def test_schedule_bookkeeping_finds_no_divergence_in_the_oracles_own_record():
    st = small_study()
    lams, xs, accs, x, p = oracle_record(st, 3, inputs.LM_ETA)
    assert accs.any() and (~accs).any()  # both decisions occur
    ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, 3, inputs.LM_ETA, lams, xs)
    assert np.all(first < 0)
    np.testing.assert_array_equal(op, p)
    np.testing.assert_array_equal(ox, x)


def test_schedule_bookkeeping_finds_a_planted_divergence():
    """Flip one voxel's decision at iteration 7 of the record (lambda x 100 or / 100 relative to
    the oracle's): it must be reported first there, with the oracle's margin and bound."""
    st = small_study()
    lams, xs, accs, *_ = oracle_record(st, 3, inputs.LM_ETA)
    k, v = 7, (0, 8, 8)
    bad = lams.copy()
    bad[k][v] *= 100.0 if accs[k][v] else 0.01
    ox, op, ol, first, margin, bound, inherited = oracle_schedule_vs_gpu(st, 3, inputs.LM_ETA, bad, xs)
    assert first[v] == k
    assert not inherited[v]
    assert np.isfinite(margin[v]) and bound[v] > 0
    # the planted voxel's neighbours read its other maps from the next iteration on: whatever they
    # do afterwards is inherited, and nothing else diverges
    others = (first >= 0) & (np.arange(first.size).reshape(first.shape) != np.ravel_multi_index(v, first.shape))
    assert np.all(first[others] > k) and np.all(inherited[others])
    assert np.count_nonzero(others) <= 8


def test_gpu_accepted_reads_lambda_moves():
    l0 = np.array([0.0, 0.0, 1.0, 1.0, 1e-8, 1e-8, 1e8])
    used = np.array([2.0, 2.0, 1.0, 1.0, 1e-8, 1e-8, 1e8])
    l1 = np.array([0.2, 20.0, 0.1, 10.0, 1e-8, 1e-7, 1e8])
    np.testing.assert_array_equal(gpu_accepted(l0, l1, used, 1e-8), [True, False, True, False, True, False, False])


def test_decision_bound_covers_model_errors_of_its_size():
    """Perturbing both model TACs by relative L2 errors of E_F (adversarially aligned with the
    residuals) moves dPhi by no more than the bound."""
    from kcs_testutil import E_F
    rng = np.random.default_rng(3)
    M = 24
    x = rng.uniform(1.0, 40.0, M)
    F0 = x * (1 + 0.1 * rng.standard_normal(M))
    F1 = x * (1 + 0.08 * rng.standard_normal(M))
    r0, r1 = x - F0, x - F1
    phi0, phi1 = 0.5 * r0 @ r0, 0.5 * r1 @ r1
    # worst case: the error of F along the residual, of norm E_F ||F||
    d0 = -E_F * np.linalg.norm(F0) * r0 / np.linalg.norm(r0)
    d1 = E_F * np.linalg.norm(F1) * r1 / np.linalg.norm(r1)
    g0, g1 = x - (F0 + d0), x - (F1 + d1)
    shift = abs((0.5 * g1 @ g1 - 0.5 * g0 @ g0) - (phi1 - phi0))
    assert shift <= decision_bound(x, phi0, phi1)
    assert shift >= 0.5 * decision_bound(x, phi0, phi1) - 2 * M * 2.0 ** -24 * (phi0 + phi1)


def test_plane_study_carries_the_whole_studys_calibration():
    """All planes of a small 3D study as a plane study: the same E_m, r_m and Huber threshold as
    the study itself; a sampled plane's expected trues are its share of the study's."""
    cfg = inputs.scaled(inputs.brain128(), nz=6, nx=48, ny=48, n_bin=48, n_ang=60, counts=1e6)
    whole = oracle.make_study(cfg)
    every = oracle.make_plane_study(cfg, range(cfg.nz))
    np.testing.assert_allclose(every.frames.E, whole.frames.E, rtol=1e-12)
    np.testing.assert_allclose(every.frames.r, whole.frames.r, rtol=1e-12)
    assert every.prior.delta == whole.prior.delta
    np.testing.assert_allclose(every.truth_x, whole.truth_x, rtol=1e-12)
    two = oracle.make_plane_study(cfg, [2, 4])
    np.testing.assert_allclose(two.frames.E, whole.frames.E, rtol=1e-12)
    np.testing.assert_array_equal(two.truth_params, whole.truth_params[:, [2, 4]])


def test_neighbour_diverged():
    from kcs_testutil import neighbour_diverged
    first = np.full((2, 5, 5), -1)
    first[0, 2, 2] = 3
    nb = neighbour_diverged(first)
    assert nb[0, 1:4, 1:4].sum() == 8 and not nb[0, 2, 2] and not nb[1].any()
    nb3 = neighbour_diverged(first, opt_nbr3d=True)
    assert nb3[1, 1:4, 1:4].all() and nb3.sum() == 8 + 9
