"""FP64 oracle: OS-MAP-OSL-KP activity update, MAP-LM kinetic fit, ICM sweep.

TEST INFRASTRUCTURE ONLY (see geometry.py).

Readings of points the paper leaves open (each is also an argument here):
  * OSL denominator (Eq. 2 with Eq. 3): Green's one-step-late form with the prior gradient
    pulling x toward the model TAC F, and sigma^2 = F / n (Poisson-like variance of the subset
    estimate), so D = n (1 + beta_kp (x - F) / max(F, eps_F)); x is unchanged where n = 0; the
    prior is off in the first sweep (no kinetic maps exist yet).
  * Expected counts add a flat background r_m (ordinary Poisson model, Sec. II-A):
    ybar = E_m P x_m + r_m with E_m = c dt_m.
  * Ordered subsets: subset q holds the angles a with a mod Q = q, processed q = 0..Q-1.
  * MAP-LM (Eq. 4-7): Levenberg damping lambda I; the Huber term uses H(t) = t^2/2 inside
    [-delta, delta] and delta |t| - delta^2/2 outside, so dH/dt = clip(t, -delta, delta); the
    3x3 in-plane neighbourhood has weight 1 for edge neighbours and 1/sqrt(2) for diagonals,
    neighbours outside the image are dropped; all voxels update synchronously from the maps of
    the previous iteration; a step is kept only if the voxel's local objective
    Phi = 1/2 ||x - F||^2 + beta_h sum_k w_k sum_p H(xi_p - xi_kp) decreases by more than
    eta Phi (eta = 0: strict decrease), then lambda /= 10 (floor lam_min), otherwise
    lambda *= 10 (cap lam_max); lambda <= 0 on entry is initialised to tau * max diag(J^T J);
    steps are clipped to the box [lo, hi].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

from . import geometry as geo
from .model import Kinetics, model_tac


@dataclass(frozen=True)
class Prior:
    beta_kp: float = 0.1
    eps_F: float = 1e-2
    beta_h: float = 0.1
    delta: Tuple[float, float, float] = (1e-3, 1e-3, 1e-3)
    kp_on: bool = True
    # 0: the in-plane 8-neighbourhood of the Huber term (the paper's prior); > 0: the 26
    # neighbours of the 3x3x3 cube with planes plane_ratio pixel sides apart (weights 1/distance)
    plane_ratio: float = 0.0


@dataclass(frozen=True)
class LMOptions:
    n_iter: int = 5
    tau: float = 1e-3
    lam_min: float = 1e-8
    lam_max: float = 1e8
    lo: Tuple[float, float, float] = (0.0, 1e-4, 0.0)
    hi: Tuple[float, float, float] = (2.0, 2.0, 1.0)
    eta: float = 0.0
    # True: every ICM sweep's fit starts its damping afresh from tau * max diag(J^T J) (the fit is
    # a new problem whenever the image has changed); False: the damping left by the previous
    # sweep's fit carries over (lambda <= 0 still means "initialise")
    restart: bool = True


@dataclass
class Frames:
    t0: np.ndarray  # minutes
    t1: np.ndarray
    E: np.ndarray  # counts per (activity unit x mm), c * dt_m
    r: np.ndarray  # background counts per bin

    @property
    def M(self) -> int:
        return len(self.t0)


# ------------------------------------------------------------------------------------------
# OS-MAP-OSL-KP
# ------------------------------------------------------------------------------------------

def subset_mult(g: geo.Geometry, mult, q: int, Q: int):
    """The multiplicative correction (attenuation x efficiency) of the rays of subset q,
    (nz, A_q, n_bin, 1), or None without one (all ones).  mult: (nz, n_ang, n_bin)."""
    if mult is None:
        return None
    return np.asarray(mult, dtype=np.float64)[:, geo.subset_angles(g.n_ang, q, Q), :, None]


def expected_counts(g: geo.Geometry, fr: Frames, x: np.ndarray, q: int, Q: int, mult=None) -> np.ndarray:
    """ybar_dm = E_m mu_d sum_v p_vd x_vm + r_m for the rays of subset q: (nz, A_q, n_bin, M);
    mu_d = 1 without a correction sinogram (the system matrix is diag(mu) P)."""
    proj = geo.forward(g, x, q, Q)
    mu = subset_mult(g, mult, q, Q)
    return fr.E * (proj if mu is None else mu * proj) + fr.r


def osl_update(g: geo.Geometry, fr: Frames, kin: Kinetics, prior: Prior, sino: np.ndarray, params: np.ndarray,
               x: np.ndarray, q: int, Q: int, kp: bool, mult=None, F=None) -> np.ndarray:
    """One OS-MAP-OSL-KP update of the image x (nz, ny, nx, M) with subset q (Eq. 2-3), with the
    system matrix diag(mult) P when a correction sinogram mult (nz, n_ang, n_bin) is given.
    F: the model TAC of `params` (shape of x), if the caller has it already (the maps do not
    change during an OSL pass, so a pass evaluates it once)."""
    ybar = expected_counts(g, fr, x, q, Q, mult)
    s_q = sino[:, geo.subset_angles(g.n_ang, q, Q)]
    ratio = np.where(ybar > 0.0, s_q / np.where(ybar > 0.0, ybar, 1.0), 0.0)
    mu = subset_mult(g, mult, q, Q)
    if mu is None:
        bp = fr.E * geo.back(g, ratio, q, Q)
        n = fr.E * geo.subset_sensitivity(g, q, Q)[None, :, :, None]
    else:
        bp = fr.E * geo.back(g, mu * ratio, q, Q)
        n = fr.E * geo.back(g, np.ascontiguousarray(mu), q, Q)  # sum_d mu_d p_vd per plane, (nz, ny, nx, 1)
    n = np.broadcast_to(n, x.shape)
    if kp:
        if F is None:
            F = model_tac(params.reshape(params.shape[0], -1).T, fr.t0, fr.t1, kin).reshape(x.shape)
        D = n * (1.0 + prior.beta_kp * (x - F) / np.maximum(F, prior.eps_F))
    else:
        D = n
    return np.where(n > 0.0, x * bp / np.where(n > 0.0, D, 1.0), x)


def initial_image(g: geo.Geometry, fr: Frames, sino: np.ndarray) -> np.ndarray:
    """Flat image per frame that reproduces the frame's net counts:
    x_m = max(sum_d (s_dm - r_m), 1) / (E_m sum_v sum_d p_vd)."""
    P = geo.system_matrix(g)
    total_p = float(P.sum()) * g.nz
    net = sino.reshape(-1, fr.M).sum(axis=0) - fr.r * (g.n_ang * g.n_bin * g.nz)
    x_m = np.maximum(net, 1.0) / (fr.E * total_p)
    return np.broadcast_to(x_m, (g.nz, g.ny, g.nx, fr.M)).copy()


# ------------------------------------------------------------------------------------------
# MAP-LM with the Huber prior
# ------------------------------------------------------------------------------------------



def huber(t, delta):
    at = np.abs(t)
    return np.where(at <= delta, 0.5 * t * t, delta * at - 0.5 * delta * delta)


def huber_grad(t, delta):
    return np.clip(t, -delta, delta)


def neighbour_offsets(plane_ratio: float = 0.0):
    """(dz, dy, dx, w) of the Huber neighbourhood: the in-plane 8-neighbours with weights 1 and
    1/sqrt(2) (Eq. 5-7), and with plane_ratio > 0 also the 18 neighbours of the adjacent planes,
    each weighted by 1 / its distance in pixel sides (planes plane_ratio pixel sides apart)."""
    dzs = (-1, 0, 1) if plane_ratio > 0 else (0,)
    out = []
    for dz in dzs:
        for dy, dx in [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]:
            if (dz, dy, dx) == (0, 0, 0):
                continue
            out.append((dz, dy, dx, 1.0 / np.sqrt(dy * dy + dx * dx + (dz * plane_ratio) ** 2)))
    return out


def _pair(d, n):
    """Slices (voxel, neighbour) along an axis of length n for offset d."""
    return (slice(0, n - d), slice(d, n)) if d >= 0 else (slice(-d, n), slice(0, n + d))


def neighbour_terms(xi_eval: np.ndarray, xi_ref: np.ndarray, delta, plane_ratio: float = 0.0
                    ) -> Tuple[np.ndarray, np.ndarray]:
    """For maps (P, nz, ny, nx): sum_k w_k psi(xi_eval_v - xi_ref_k) per parameter (P, ...) and
    sum_k w_k sum_p H(xi_eval_vp - xi_ref_kp) (nz, ny, nx) over the neighbours k of
    neighbour_offsets(plane_ratio) that lie inside the image."""
    _, nz, ny, nx = xi_ref.shape
    grad = np.zeros_like(xi_eval)
    energy = np.zeros(xi_eval.shape[1:])
    for dz, dy, dx, w in neighbour_offsets(plane_ratio):
        (zs, zd), (ys, yd), (xs, xd) = _pair(dz, nz), _pair(dy, ny), _pair(dx, nx)
        # voxel at (z, y, x) = source slices; its neighbour at (z+dz, y+dy, x+dx) = destination slices
        for p in range(xi_ref.shape[0]):
            t = xi_eval[p][zs, ys, xs] - xi_ref[p][zd, yd, xd]
            grad[p][zs, ys, xs] += w * huber_grad(t, delta[p])
            energy[zs, ys, xs] += w * huber(t, delta[p])
    return grad, energy


def lm_iteration(fr: Frames, kin: Kinetics, prior: Prior, opt: LMOptions, x: np.ndarray, params: np.ndarray,
                 lam: np.ndarray, with_objective: bool = False):
    """One synchronous MAP-LM iteration over all voxels (Eq. 4).  x: (nz, ny, nx, M);
    params: (P, nz, ny, nx), P = 3 maps (K1, k2, k3) or 4 (with the blood fraction vb); prior.delta,
    opt.lo and opt.hi hold P entries; lam: (nz, ny, nx).  Returns new (params, lam), followed by
    the voxel objectives before and at the trial step (phi0, phi1), each (nz, ny, nx), when
    `with_objective` is set."""
    n_par = params.shape[0]
    shp = params.shape[1:]
    N = int(np.prod(shp))
    xv = x.reshape(N, -1)
    xi = params.reshape(n_par, N).T.copy()
    F, J = model_tac(xi, fr.t0, fr.t1, kin, jacobian=True)
    r = xv - F
    pg, pe = neighbour_terms(params, params, prior.delta, prior.plane_ratio)
    g = np.einsum("nmp,nm->np", J, r) - prior.beta_h * pg.reshape(n_par, N).T
    A = np.einsum("nmp,nmq->npq", J, J)
    lam = lam.reshape(N).copy()
    init = lam <= 0.0
    lam[init] = opt.tau * np.max(np.diagonal(A, axis1=1, axis2=2), axis=1)[init]
    step = np.linalg.solve(A + lam[:, None, None] * np.eye(n_par)[None], g[:, :, None])[:, :, 0]
    trial = np.clip(xi + step, np.array(opt.lo), np.array(opt.hi))
    F1 = model_tac(trial, fr.t0, fr.t1, kin)
    trial_maps = trial.T.reshape(params.shape)
    _, pe1 = neighbour_terms(trial_maps, params, prior.delta, prior.plane_ratio)
    phi0 = 0.5 * np.sum(r * r, axis=1) + prior.beta_h * pe.reshape(N)
    phi1 = 0.5 * np.sum((xv - F1) ** 2, axis=1) + prior.beta_h * pe1.reshape(N)
    accept = phi1 - phi0 < -opt.eta * phi0
    new = np.where(accept[:, None], trial, xi)
    lam = np.where(accept, np.maximum(lam / 10.0, opt.lam_min), np.minimum(lam * 10.0, opt.lam_max))
    out = (new.T.reshape(params.shape).copy(), lam.reshape(shp))
    return out + (phi0.reshape(shp), phi1.reshape(shp)) if with_objective else out


def lm_fit(fr, kin, prior, opt, x, params, lam):
    for _ in range(opt.n_iter):
        params, lam = lm_iteration(fr, kin, prior, opt, x, params, lam)
    return params, lam


# ------------------------------------------------------------------------------------------
# ICM
# ------------------------------------------------------------------------------------------

def icm_sweep(g, fr, kin, prior, opt, sino, x, params, lam, Q: int, sweep_idx: int, mult=None):
    """One ICM sweep (Sec. II-D): OS-MAP-OSL-KP over all Q subsets given the maps, then MAP-LM
    given the new image.  With opt.restart (the default) each sweep's MAP-LM is a new fit to a
    new image and its damping starts from tau * max diag(J^T J) (the lambda passed in is
    ignored); otherwise it continues from the lambda passed in.  The final lambda is returned."""
    kp = prior.kp_on and sweep_idx > 0
    F = model_tac(params.reshape(params.shape[0], -1).T, fr.t0, fr.t1, kin).reshape(x.shape) if kp else None
    for q in range(Q):
        x = osl_update(g, fr, kin, prior, sino, params, x, q, Q, kp, mult, F)
    params, lam = lm_fit(fr, kin, prior, opt, x, params, np.zeros_like(lam) if opt.restart else lam)
    return x, params, lam


def initial_state(g: geo.Geometry, fr: Frames, sino: np.ndarray, xi0=(0.08, 0.12, 0.05)):
    """Flat image, maps xi0 everywhere (3 values, or 4 with the blood fraction), lambda 0."""
    x = initial_image(g, fr, sino)
    params = np.empty((len(xi0), g.nz, g.ny, g.nx))
    for p in range(len(xi0)):
        params[p] = xi0[p]
    lam = np.zeros((g.nz, g.ny, g.nx))
    return x, params, lam


def icm(g, fr, kin, prior, opt, sino, Q: int, n_sweeps: int, state=None, mult=None):
    """n_sweeps ICM sweeps from the initial state (the flat start ignores mult: the first OSL
    update rescales the image to the data)."""
    x, params, lam = state if state is not None else initial_state(g, fr, sino)
    for s in range(n_sweeps):
        x, params, lam = icm_sweep(g, fr, kin, prior, opt, sino, x, params, lam, Q, s, mult)
    return x, params, lam
