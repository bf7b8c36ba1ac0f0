"""Whole-schedule behaviour of the oracle ICM (Sec. II-D) on noise-free 64x64 data: the paper
prints no numbers, so the pins are invariants and convergence toward the known truth."""
import numpy as np

import oracle
from paper_1803_10045_amd import inputs


def test_noise_free_icm_moves_toward_truth():
    cfg = inputs.disk64()
    st = oracle.make_study(cfg)
    clean = st.frames.E * oracle.forward(st.geom, st.truth_x) + st.frames.r
    state = oracle.initial_state(st.geom, st.frames, clean)
    errs = []
    for s in range(cfg.n_sweeps):
        state = oracle.icm_sweep(st.geom, st.frames, st.kin, st.prior, st.lm, clean, *state, cfg.Q, s)
        x, p, lam = state
        assert np.all(x >= 0)
        lo, hi = np.array(inputs.LM_LO), np.array(inputs.LM_HI)
        assert np.all(p >= lo[:, None, None, None]) and np.all(p <= hi[:, None, None, None])
        errs.append(np.linalg.norm(x - st.truth_x) / np.linalg.norm(st.truth_x))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.3 * errs[0]
    wm = st.truth_params[0] == inputs.WHITE[0]
    for k in range(3):
        assert abs(np.median(p[k][wm]) / inputs.WHITE[k] - 1) < 0.05
