"""Pins of the oracle's kinetic model against independent numerics (ODE solver, quadrature,
closed forms, finite differences)."""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

import oracle
from paper_1803_10045_amd import inputs

KIN = oracle.Kinetics(**inputs.FENG, vb=inputs.VB)
T0, T1 = inputs.frame_times()


def ode_frames(p, t0=T0, t1=T1, kin=KIN):
    """Frame averages from a DOP853 solve of the compartment ODEs plus running integrals."""
    K1, k2, k3 = p

    def f(t, y):
        c = float(oracle.cp(t, kin))
        C1, C2 = y[0], y[1]
        return [K1 * c - (k2 + k3) * C1, k3 * C1, C1 + C2, c]

    tb = np.unique(np.concatenate([t0, t1]))
    sol = solve_ivp(f, (0.0, tb[-1]), [0.0, 0.0, 0.0, 0.0], method="DOP853", rtol=1e-12, atol=1e-13,
                    t_eval=tb)
    ict = dict(zip(tb, sol.y[2]))
    icp = dict(zip(tb, sol.y[3]))
    return np.array([((1 - kin.vb) * (ict[b] - ict[a]) + kin.vb * (icp[b] - icp[a])) / (b - a)
                     for a, b in zip(t0, t1)])


def test_feng_input_at_zero_and_total_area():
    assert oracle.cp(0.0, KIN) == pytest.approx(0.0, abs=1e-12)
    assert oracle.cp(-1.0, KIN) == 0.0
    # int_0^inf Cp = A1/l1^2 + (A2+A3)/l1 - A2/l2 - A3/l3 (termwise integrals of the exponentials)
    k = KIN
    closed = k.A1 / k.l1 ** 2 + (k.A2 + k.A3) / k.l1 - k.A2 / k.l2 - k.A3 / k.l3
    P1, _ = oracle.input_integrals(np.array([1e4]), KIN)
    assert P1[0] == pytest.approx(closed, rel=1e-12)


@pytest.mark.parametrize("T", [0.05, 0.3, 1.0, 5.0, 17.5, 40.0])
def test_input_integrals_against_quadrature(T):
    P1, P2 = oracle.input_integrals(np.array([T]), KIN)
    q1 = quad(lambda t: oracle.cp(t, KIN), 0, T, epsabs=0, epsrel=1e-13, limit=200)[0]
    # P2 = int_0^T (T - s) Cp(s) ds (Cauchy's formula for repeated integration)
    q2 = quad(lambda t: (T - t) * oracle.cp(t, KIN), 0, T, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert P1[0] == pytest.approx(q1, rel=1e-11)
    assert P2[0] == pytest.approx(q2, rel=1e-11)


def test_moments_against_quadrature():
    for z in [-150.0, -20.0, -1.0, -0.999, -0.3, -1e-9, 0.0, 1e-6, 0.5, 0.999, 1.0, 3.0, 60.0]:
        m = oracle.moments(np.array([z]), 3)[:, 0]
        for k in range(4):
            ref = quad(lambda s: s ** k * np.exp(z * s), 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
            assert m[k] == pytest.approx(ref, rel=1e-12), (z, k)


PARAMS = [inputs.WHITE, inputs.GRAY, inputs.HOT,
          (0.75, 0.35, 0.031), (0.51, 0.27, 0.018),  # simulation table rows (Table I)
          (0.102 * 0.7, 0.130 * 1.3, 0.062 * 0.7), (0.2, 1e-4, 0.0), (0.05, 2.0, 1.0), (1.0, 1e-4, 1e-3)]


@pytest.mark.parametrize("p", PARAMS)
def test_frame_tacs_against_ode(p):
    F = oracle.model_tac(np.array(p), T0, T1, KIN)[0]
    ref = ode_frames(p)
    np.testing.assert_allclose(F, ref, rtol=2e-9, atol=0)


def test_known_tac_values():
    # frame 0 / frame 23 of the white-matter, gray-matter and hot classes (BJ schedule, vb = 0.05),
    # cross-checked here against the ODE solution rather than stored
    F = oracle.model_tac(np.array([inputs.WHITE, inputs.GRAY, inputs.HOT]), T0, T1, KIN)
    for i, p in enumerate([inputs.WHITE, inputs.GRAY, inputs.HOT]):
        ref = ode_frames(p)
        assert F[i, 0] == pytest.approx(ref[0], rel=1e-9)
        assert F[i, -1] == pytest.approx(ref[-1], rel=1e-9)
    assert F[0, 0] == pytest.approx(3.030, abs=1e-3) and F[0, -1] == pytest.approx(17.450, abs=1e-3)


@pytest.mark.parametrize("lam_name", ["l1", "l2", "l3"])
def test_removable_singularity(lam_name):
    """k2 + k3 = -lambda_i makes the convolution of that exponential degenerate (0/0);
    the model must stay continuous and match the ODE there."""
    lam = getattr(KIN, lam_name)
    a0 = -lam
    if a0 > 3.0:  # outside the parameter box
        pytest.skip("k2 + k3 = 4.134 lies outside the bounds")
    for eps in [0.0, 1e-15, 1e-12, 1e-9, 1e-6, 1e-3, -1e-6, -1e-3]:
        a = a0 + eps
        p = (0.1, 0.6 * a, 0.4 * a)
        F = oracle.model_tac(np.array(p), T0, T1, KIN)[0]
        np.testing.assert_allclose(F, ode_frames(p), rtol=2e-9)


@pytest.mark.parametrize("p", [inputs.WHITE, inputs.GRAY, inputs.HOT, (0.3, 0.1191, 0.0), (0.1, 0.02, 0.00043)])
def test_jacobian_against_central_differences(p):
    p = np.array(p, dtype=np.float64)
    F, J = oracle.model_tac(p, T0, T1, KIN, jacobian=True)
    for k in range(3):
        h = 1e-6 * max(abs(p[k]), 0.05)
        dp = np.zeros(3)
        dp[k] = h
        fd = (oracle.model_tac(p + dp, T0, T1, KIN) - oracle.model_tac(p - dp, T0, T1, KIN))[0] / (2 * h)
        scale = np.max(np.abs(J[0, :, k])) + 1e-30
        assert np.max(np.abs(fd - J[0, :, k])) / scale < 1e-7, k


def test_special_cases_of_the_tissue_model():
    # k2 -> 0: all tracer that enters is trapped, int_0^T C_T = K1 int_0^T P1 = K1 P2
    T = np.array([0.5, 3.0, 40.0])
    C, _ = oracle.cumulative_tissue(np.array([[0.3, 1e-13, 0.05]]), T, KIN)
    _, P2 = oracle.input_integrals(T, KIN)
    np.testing.assert_allclose(C[0], 0.3 * P2, rtol=1e-10)
    # k3 = 0: one reversible compartment, C_T = K1 e^{-k2 t} (*) Cp
    K1, k2 = 0.2, 0.15
    C, _ = oracle.cumulative_tissue(np.array([[K1, k2, 0.0]]), T, KIN)
    for i, t in enumerate(T):
        ct = lambda u: K1 * quad(lambda s: oracle.cp(s, KIN) * np.exp(-k2 * (u - s)), 0, u, epsrel=1e-13,
                                 limit=200)[0]
        ref = quad(ct, 0, t, epsrel=1e-11, limit=200)[0]
        assert C[0, i] == pytest.approx(ref, rel=1e-9)
    # linear in K1
    C1, _ = oracle.cumulative_tissue(np.array([[0.1, 0.1, 0.05]]), T, KIN)
    C2, _ = oracle.cumulative_tissue(np.array([[0.3, 0.1, 0.05]]), T, KIN)
    np.testing.assert_allclose(C2, 3 * C1, rtol=1e-13)


@pytest.mark.parametrize("p", [(0.10, 0.10, 0.05), (0.30, 0.02, 0.40), (0.05, 0.90, 0.01), (0.20, 0.0, 0.07),
                               (0.15, 0.12, 0.0), (0.25, 0.0, 0.0)])
def test_net_influx_is_the_late_slope_for_a_constant_input(p):
    """K_i pinned to the compartment model itself: under a constant unit plasma input the tissue
    curve of the irreversible model becomes a straight line of slope K_i (DOP853 solve of the
    ODEs; with k2 + k3 = 0 the first compartment just fills at rate K1)."""
    K1, k2, k3 = p
    a = k2 + k3

    def f(t, c):
        return [K1 - a * c[0], k3 * c[0]]

    T1, T2 = (40.0 / a, 80.0 / a) if a > 0 else (10.0, 20.0)
    sol = solve_ivp(f, (0.0, T2), [0.0, 0.0], method="DOP853", rtol=1e-12, atol=1e-14, t_eval=[T1, T2],
                    dense_output=False)
    ct = sol.y[0] + sol.y[1]
    slope = (ct[1] - ct[0]) / (T2 - T1)
    ki = oracle.net_influx(np.array(p, dtype=np.float64).reshape(3, 1))[0]
    assert ki == pytest.approx(slope, rel=1e-9, abs=1e-12)


def test_net_influx_shapes_and_limits():
    p = np.array([[[0.2, 0.3]], [[0.1, 1e-12]], [[0.05, 0.2]]])  # [3, 1, 2]
    ki = oracle.net_influx(p)
    assert ki.shape == (1, 2)
    np.testing.assert_allclose(ki[0], [0.2 * 0.05 / 0.15, 0.3 * 0.2 / (0.2 + 1e-12)], rtol=1e-15)


# ---------------------------------------------------------------------------------------------
# The blood fraction as a fourth fitted parameter (the paper's f_v map, Sec. IV and Table I):
# params (K1, k2, k3, vb) with vb per voxel.

def kin_with_vb(vb):
    import dataclasses
    return dataclasses.replace(KIN, vb=float(vb))


@pytest.mark.parametrize("p", [(0.102, 0.130, 0.062, 0.0), (0.054, 0.109, 0.045, 0.03), (0.12, 0.10, 0.12, 0.3),
                               (0.0, 0.12, 0.05, 1.0), (0.75, 0.35, 0.031, 0.13)])
def test_frame_tacs_with_free_blood_fraction_against_ode(p):
    """F with vb taken from the fourth parameter equals the ODE frames with that blood fraction
    (and ignores the Kinetics' own vb)."""
    p = np.array(p)
    F = oracle.model_tac(p, T0, T1, kin_with_vb(0.77))[0]
    np.testing.assert_allclose(F, ode_frames(p[:3], kin=kin_with_vb(p[3])), rtol=2e-9, atol=1e-12)


@pytest.mark.parametrize("p", [(0.102, 0.130, 0.062, 0.05), (0.054, 0.109, 0.045, 0.2), (0.3, 0.1191, 0.01, 0.6)])
def test_four_parameter_jacobian_against_ode_differences(p):
    """All four columns against central differences of the ODE frames (h = 1e-6 relative); the
    vb column is exact for a difference since F is linear in vb."""
    p = np.array(p, dtype=np.float64)
    _, J = oracle.model_tac(p, T0, T1, KIN, jacobian=True)
    assert J.shape == (1, len(T0), 4)
    for k in range(4):
        h = 1e-6 * max(abs(p[k]), 0.05)
        dp = np.zeros(4)
        dp[k] = h
        hi, lo = p + dp, p - dp
        fd = (ode_frames(hi[:3], kin=kin_with_vb(hi[3])) - ode_frames(lo[:3], kin=kin_with_vb(lo[3]))) / (2 * h)
        scale = np.max(np.abs(J[0, :, k]))
        assert np.max(np.abs(fd - J[0, :, k])) / scale < 1e-6, k


def test_three_parameter_calls_keep_the_fixed_blood_fraction():
    p3 = np.array(inputs.GRAY)
    p4 = np.append(p3, KIN.vb)
    F3, J3 = oracle.model_tac(p3, T0, T1, KIN, jacobian=True)
    F4, J4 = oracle.model_tac(p4, T0, T1, KIN, jacobian=True)
    np.testing.assert_allclose(F4, F3, rtol=1e-14)
    np.testing.assert_allclose(J4[..., :3], J3, rtol=1e-14)
