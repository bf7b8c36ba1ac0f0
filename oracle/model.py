"""FP64 oracle: plasma input, irreversible two-tissue model, frame-averaged TACs and Jacobian.

TEST INFRASTRUCTURE ONLY (see geometry.py).

Kinetic model (Sec. II-C, Eq. 3-4; model named in Sec. III-A and IV-A): irreversible two-tissue
compartments with K1, k2, k3 (k4 = 0) and a fixed blood fraction vb,

    dC1/dt = K1 Cp - (k2 + k3) C1,   dC2/dt = k3 C1,   C_T = C1 + C2,
    C_PET(t) = (1 - vb) C_T(t) + vb Cp(t).

With a = k2 + k3 the impulse response of the tissue is K1 (k3 + k2 e^{-a t}) / a, so the
running integral of C_T is

    int_0^T C_T = K1 [ alpha P2(T) + (1 - alpha) I(T) ],   alpha = k3 / a,

where P1 = int_0^T Cp, P2 = int_0^T P1 and I = int_0^T G with G = Cp (*) e^{-a t}
(convolution).  From G' = Cp - a G, I = (P1 - G) / a.  The frame value is the frame average
F_m = (1/dt_m) int_{t0_m}^{t1_m} C_PET dt (time integrals of the model, Sec. II-C), evaluated
in closed form: no numerical integration.

The plasma input is the Feng model Cp(t) = (A1 t - A2 - A3) e^{l1 t} + A2 e^{l2 t} + A3 e^{l3 t}
(t >= 0, in minutes), i.e. a sum of components c t^n e^{l t} with n in {0, 1}.  Every integral
above is, per component, a moment m_k(z) = int_0^1 s^k e^{z s} ds of an exponential, evaluated
by its power series for |z| < 1 and by the recursion m_k = (e^z - k m_{k-1}) / z otherwise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Kinetics:
    A1: float = 851.1
    A2: float = 21.88
    A3: float = 20.81
    l1: float = -4.134
    l2: float = -0.1191
    l3: float = -0.01043
    vb: float = 0.05

    def components(self):
        """Feng input as (coefficient, rate, power) triples: Cp = sum c t^n e^{l t}."""
        return ((self.A1, self.l1, 1), (-(self.A2 + self.A3), self.l1, 0), (self.A2, self.l2, 0),
                (self.A3, self.l3, 0))


def cp(t, kin: Kinetics) -> np.ndarray:
    """Feng plasma input; 0 for t < 0."""
    t = np.asarray(t, dtype=np.float64)
    tt = np.maximum(t, 0.0)
    v = (kin.A1 * tt - kin.A2 - kin.A3) * np.exp(kin.l1 * tt) + kin.A2 * np.exp(kin.l2 * tt) + kin.A3 * np.exp(kin.l3 * tt)
    return np.where(t >= 0.0, v, 0.0)


def moments(z, kmax: int) -> np.ndarray:
    """m_k(z) = int_0^1 s^k e^{z s} ds for k = 0..kmax (stacked on axis 0)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty((kmax + 1,) + z.shape)
    small = np.abs(z) < 1.0
    zs = z[small]
    term = np.ones_like(zs)  # z^j / j!
    acc = [np.zeros_like(zs) for _ in range(kmax + 1)]
    for j in range(26):  # m_k = sum_j z^j / (j! (j + k + 1))
        for k in range(kmax + 1):
            acc[k] += term / (j + k + 1)
        term = term * zs / (j + 1)
    zb = z[~small]
    ez = np.exp(zb)
    m = np.expm1(zb) / zb  # m_0; then m_k = (e^z - k m_{k-1}) / z
    for k in range(kmax + 1):
        if k > 0:
            m = (ez - k * m) / zb
        out[k][small] = acc[k]
        out[k][~small] = m
    return out


def input_integrals(T, kin: Kinetics):
    """P1(T) = int_0^T Cp and P2(T) = int_0^T P1, for an array of times T >= 0."""
    T = np.asarray(T, dtype=np.float64)
    P1 = np.zeros_like(T)
    P2 = np.zeros_like(T)
    for c, lam, n in kin.components():
        m = moments(lam * T, n + 1)
        P1 = P1 + c * T ** (n + 1) * m[n]
        P2 = P2 + c * T ** (n + 2) * (m[n] - m[n + 1])
    return P1, P2


def cumulative_tissue(params: np.ndarray, T: np.ndarray, kin: Kinetics, jacobian: bool = False):
    """int_0^T C_T for each voxel (rows of params = (K1, k2, k3)) and each time T.

    Returns C (n, nT) and, if requested, dC/d(K1, k2, k3) as (n, nT, 3).  The convolutions of
    the input with e^{-a t} and t e^{-a t} (a = k2 + k3) and the combination above are evaluated
    per voxel and time in ``kinetics.c`` (same closed form, FP64, OpenMP over voxels); P1 and P2
    come from :func:`input_integrals`."""
    from .geometry import _lib

    params = np.ascontiguousarray(np.atleast_2d(np.asarray(params, dtype=np.float64)))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64).ravel())
    if np.any(params[:, 1] + params[:, 2] <= 0.0):
        raise ValueError("k2 + k3 must be positive")
    P1, P2 = input_integrals(T, kin)
    comp = np.array(kin.components(), dtype=np.float64).ravel()
    n, nT = params.shape[0], T.shape[0]
    C = np.empty((n, nT))
    D = np.empty((n, nT, 3)) if jacobian else None
    _lib().orc_tissue_integrals(n, params, nT, T, np.ascontiguousarray(P1), np.ascontiguousarray(P2),
                                len(kin.components()), comp, C, None if D is None else D.ctypes.data)
    return C, D


def model_tac(params: np.ndarray, t0: np.ndarray, t1: np.ndarray, kin: Kinetics, jacobian: bool = False,
              chunk: int = 1 << 18):
    """Frame-averaged model TAC F_m(xi) (n, M) and optionally its Jacobian (n, M, P).

    params: (n, 3) rows (K1, k2, k3) with the blood fraction kin.vb, or (n, 4) rows
    (K1, k2, k3, vb) with a blood fraction per voxel (the paper's f_v fitted as a fourth map,
    Sec. IV and Table I).  F_m = [(1 - vb) int_frame C_T + vb int_frame Cp] / dt_m, so the
    derivative by vb is (int_frame Cp - int_frame C_T) / dt_m."""
    params = np.atleast_2d(np.asarray(params, dtype=np.float64))
    n_par = params.shape[1]
    if n_par not in (3, 4):
        raise ValueError("params must have 3 or 4 columns")
    t0 = np.asarray(t0, dtype=np.float64)
    t1 = np.asarray(t1, dtype=np.float64)
    dt = t1 - t0
    P1_0, _ = input_integrals(t0, kin)
    P1_1, _ = input_integrals(t1, kin)
    cp_int = P1_1 - P1_0  # int_frame Cp
    n = params.shape[0]
    M = len(t0)
    F = np.empty((n, M))
    J = np.empty((n, M, n_par)) if jacobian else None
    tb, inv = np.unique(np.concatenate([t0, t1]), return_inverse=True)
    i0, i1 = inv[:M], inv[M:]
    for s in range(0, n, chunk):
        p = params[s:s + chunk]
        vb = p[:, 3:4] if n_par == 4 else kin.vb
        C, D = cumulative_tissue(np.ascontiguousarray(p[:, :3]), tb, kin, jacobian)
        tissue = np.take(C, i1, axis=1) - np.take(C, i0, axis=1)  # int_frame C_T
        F[s:s + chunk] = ((1.0 - vb) * tissue + vb * cp_int[None, :]) / dt[None, :]
        if jacobian:
            vbj = vb[:, :, None] if n_par == 4 else vb
            J[s:s + chunk, :, :3] = (1.0 - vbj) * (np.take(D, i1, axis=1) - np.take(D, i0, axis=1)) / dt[None, :, None]
            if n_par == 4:
                J[s:s + chunk, :, 3] = (cp_int[None, :] - tissue) / dt[None, :]
    return (F, J) if jacobian else F


def net_influx(params: np.ndarray) -> np.ndarray:
    """Macro-parameter K_i = K1 k3 / (k2 + k3) of the irreversible model (Sec. IV, human data):
    the net uptake rate, the late slope of the tissue response to a constant unit input.  Where
    k2 + k3 = 0 nothing leaves the first compartment and K_i = K1.  params: [3, ...]."""
    K1, k2, k3 = (np.asarray(params[i], dtype=np.float64) for i in range(3))
    a = k2 + k3
    pos = a > 0
    return np.where(pos, K1 * k3 / np.where(pos, a, 1.0), K1)
