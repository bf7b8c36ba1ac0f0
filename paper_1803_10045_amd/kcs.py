"""Python binding of libkcs (include/kcs.h): argument marshalling only.

Every function here has the name of the C entry point it calls and forwards device pointers of
FP32 torch tensors plus the current torch stream; all arithmetic happens in the HIP library.
If the library is not built the import of any entry point raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from functools import lru_cache
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkcs.so")

KCS_OK, KCS_EINVAL, KCS_ESHAPE, KCS_EWORKSPACE, KCS_EHIP = 0, -1, -2, -3, -4

# Entry points declared in include/kcs.h (checked against the header by the tests).
ENTRY_POINTS = ("kcs_workspace_bytes", "kcs_study_footprint_bytes", "kcs_project", "kcs_backproject",
                "kcs_model_tac", "kcs_ki_map", "kcs_rebin_ssrb", "kcs_osl_update", "kcs_lm_fit", "kcs_init_state", "kcs_icm_sweep",
                "kcs_icm_sweep_noalloc",
                "kcs_plan_create", "kcs_plan_run", "kcs_plan_describe", "kcs_plan_destroy",
                "kcs_timing_enable", "kcs_timing_collect", "kcs_stream_probe", "kcs_last_error")

KCS_PLAN_GRAPH, KCS_PLAN_AUTOTUNE = 1, 2

TIMING_KINDS = ("setup", "project", "back", "osl", "lm", "model", "init", "copy")


class KcsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kcs error {code}: {msg}")
        self.code = code


class c_geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
                ("n_ang", ctypes.c_int32), ("n_bin", ctypes.c_int32), ("bin_mm", ctypes.c_double),
                ("ang0_rad", ctypes.c_double), ("d_mult", ctypes.c_void_p)]


_dp = ctypes.POINTER(ctypes.c_double)


class c_frames(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("t0_min", _dp), ("t1_min", _dp), ("scale", _dp), ("bg", _dp)]


class c_kinetics(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("A1", "A2", "A3", "l1", "l2", "l3", "vb")] + [("fit_vb", ctypes.c_int32)]


class c_prior(ctypes.Structure):
    _fields_ = [("beta_kp", ctypes.c_double), ("eps_F", ctypes.c_double), ("beta_h", ctypes.c_double),
                ("delta", ctypes.c_double * 4), ("kp_on", ctypes.c_int32), ("plane_ratio", ctypes.c_double)]


class c_lm_opts(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("tau", ctypes.c_double), ("lam_min", ctypes.c_double),
                ("lam_max", ctypes.c_double), ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4),
                ("eta", ctypes.c_double), ("restart", ctypes.c_int32)]


class c_study(ctypes.Structure):
    _fields_ = [("g", c_geometry), ("f", c_frames), ("k", c_kinetics), ("p", c_prior), ("lm", c_lm_opts),
                ("Q", ctypes.c_int32), ("sweep_begin", ctypes.c_int32), ("sweep_end", ctypes.c_int32),
                ("d_sino", ctypes.c_void_p), ("d_x", ctypes.c_void_p), ("d_params", ctypes.c_void_p),
                ("d_lambda", ctypes.c_void_p), ("d_work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


@lru_cache(maxsize=1)
def lib() -> ctypes.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1803_10045_amd/build.py")
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    L.kcs_workspace_bytes.argtypes = [P(c_geometry), i32, i32]
    L.kcs_workspace_bytes.restype = sz
    L.kcs_study_footprint_bytes.argtypes = [P(c_geometry), i32, i32]
    L.kcs_study_footprint_bytes.restype = sz
    L.kcs_project.argtypes = [P(c_geometry), P(c_frames), vp, i32, i32, vp, vp]
    L.kcs_backproject.argtypes = [P(c_geometry), P(c_frames), vp, i32, i32, vp, vp, vp]
    L.kcs_model_tac.argtypes = [P(c_frames), P(c_kinetics), vp, i64, vp, vp, vp, sz, vp]
    L.kcs_ki_map.argtypes = [vp, i64, vp, vp]
    L.kcs_rebin_ssrb.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp]
    L.kcs_osl_update.argtypes = [P(c_geometry), P(c_frames), P(c_kinetics), P(c_prior), vp, vp, i32, i32, vp, vp, sz,
                                 vp]
    L.kcs_lm_fit.argtypes = [P(c_geometry), P(c_frames), P(c_kinetics), P(c_prior), P(c_lm_opts), vp, vp, vp, vp, sz,
                             vp]
    L.kcs_init_state.argtypes = [P(c_geometry), P(c_frames), vp, P(ctypes.c_double), i32, vp, vp, vp, vp, sz, vp]
    L.kcs_icm_sweep.argtypes = [P(c_geometry), P(c_frames), P(c_kinetics), P(c_prior), P(c_lm_opts), vp, i32, i32, vp,
                                vp, vp, vp, sz, vp]
    L.kcs_icm_sweep_noalloc.argtypes = [P(c_geometry), P(c_frames), P(c_kinetics), P(c_prior), P(c_lm_opts), vp, i32,
                                        i32, vp, vp, vp, vp]
    for name in ("kcs_project", "kcs_backproject", "kcs_model_tac", "kcs_ki_map", "kcs_rebin_ssrb", "kcs_osl_update",
                 "kcs_lm_fit",
                 "kcs_init_state", "kcs_icm_sweep", "kcs_icm_sweep_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    L.kcs_plan_create.argtypes = [P(c_study), i32, i32, vp, P(vp)]
    L.kcs_plan_create.restype = ctypes.c_int
    L.kcs_plan_run.argtypes = [vp, vp]
    L.kcs_plan_run.restype = ctypes.c_int
    L.kcs_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.kcs_plan_describe.restype = ctypes.c_int
    L.kcs_plan_destroy.argtypes = [vp]
    L.kcs_plan_destroy.restype = None
    L.kcs_timing_enable.argtypes = [i32]
    L.kcs_timing_enable.restype = ctypes.c_int
    L.kcs_timing_collect.argtypes = [P(ctypes.c_double), P(ctypes.c_int64)]
    L.kcs_timing_collect.restype = ctypes.c_int
    L.kcs_stream_probe.argtypes = [i32, vp, vp, sz, i32, vp]
    L.kcs_stream_probe.restype = ctypes.c_int
    L.kcs_last_error.argtypes = []
    L.kcs_last_error.restype = ctypes.c_char_p
    return L


# ----------------------------------------------------------------------------------------------
# Host-side argument objects
# ----------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    nz: int
    pixel_mm: float
    n_ang: int
    n_bin: int
    bin_mm: float
    ang0_rad: float = 0.0
    # multiplicative correction sinogram (attenuation x efficiency) [nz][n_ang][n_bin], a float32
    # device tensor, or None for all ones
    mult: Optional[object] = field(default=None, compare=False, hash=False, repr=False)

    @classmethod
    def from_config(cls, cfg) -> "Geometry":
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.pixel_mm, cfg.n_ang, cfg.n_bin, cfg.bin_mm, cfg.ang0)

    def c(self) -> c_geometry:
        return c_geometry(self.nx, self.ny, self.nz, self.pixel_mm, self.n_ang, self.n_bin, self.bin_mm, self.ang0_rad,
                          _ptr(self.mult, (self.nz, self.n_ang, self.n_bin), "mult"))

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    def subset_size(self, q: int, Q: int) -> int:
        return (self.n_ang - q + Q - 1) // Q


class Frames:
    """Frame schedule (minutes) with per-frame scale E_m and background r_m (FP64 host arrays)."""

    def __init__(self, t0, t1, scale, bg):
        self.t0 = np.ascontiguousarray(t0, dtype=np.float64)
        self.t1 = np.ascontiguousarray(t1, dtype=np.float64)
        self.scale = np.ascontiguousarray(scale, dtype=np.float64)
        self.bg = np.ascontiguousarray(bg, dtype=np.float64)
        n = len(self.t0)
        if not (len(self.t1) == len(self.scale) == len(self.bg) == n):
            raise ValueError("frame arrays must have equal length")

    @property
    def M(self) -> int:
        return len(self.t0)

    def c(self) -> c_frames:
        p = lambda a: a.ctypes.data_as(_dp)
        return c_frames(self.M, p(self.t0), p(self.t1), p(self.scale), p(self.bg))


@dataclass(frozen=True)
class Kinetics:
    A1: float
    A2: float
    A3: float
    l1: float
    l2: float
    l3: float
    vb: float
    fit_vb: bool = False  # True: the blood fraction is a fourth map (maps [4][...]), vb unused

    @property
    def n_maps(self) -> int:
        return 4 if self.fit_vb else 3

    def c(self) -> c_kinetics:
        return c_kinetics(self.A1, self.A2, self.A3, self.l1, self.l2, self.l3, self.vb, int(self.fit_vb))


@dataclass(frozen=True)
class Prior:
    beta_kp: float
    eps_F: float
    beta_h: float
    delta: Sequence[float]
    kp_on: bool = True
    plane_ratio: float = 0.0  # 0: in-plane 3x3 neighbourhood; > 0: 3x3x3, planes this many pixel sides apart

    def c(self) -> c_prior:
        d = tuple(self.delta) + (tuple(self.delta)[-1],) * (4 - len(self.delta))  # 3 maps: delta[3] unused
        return c_prior(self.beta_kp, self.eps_F, self.beta_h, (ctypes.c_double * 4)(*d), int(self.kp_on),
                       float(self.plane_ratio))


@dataclass(frozen=True)
class LMOptions:
    n_iter: int
    tau: float
    lam_min: float
    lam_max: float
    lo: Sequence[float]
    hi: Sequence[float]
    eta: float = 0.0
    restart: bool = True  # ICM sweeps: every sweep's fit starts lambda afresh (False: carries it over)

    def c(self) -> c_lm_opts:
        lo = tuple(self.lo) + (0.0,) * (4 - len(self.lo))  # blood-fraction bounds, read with fit_vb only
        hi = tuple(self.hi) + (1.0,) * (4 - len(self.hi))
        return c_lm_opts(self.n_iter, self.tau, self.lam_min, self.lam_max, (ctypes.c_double * 4)(*lo),
                         (ctypes.c_double * 4)(*hi), self.eta, int(self.restart))


# ----------------------------------------------------------------------------------------------
# Marshalling helpers
# ----------------------------------------------------------------------------------------------

def _stream(stream) -> ctypes.c_void_p:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, shape=None, name="tensor", dtype=None) -> ctypes.c_void_p:
    import torch
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    want = torch.float32 if dtype is None else dtype
    if t.dtype != want:
        raise ValueError(f"{name} must be {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _check(rc: int):
    if rc != KCS_OK:
        raise KcsError(rc, lib().kcs_last_error().decode())


def _work(w):
    import torch
    if w is None or not w.is_cuda or w.dtype != torch.uint8:
        raise ValueError("workspace must be a uint8 device tensor")
    return ctypes.c_void_p(w.data_ptr()), ctypes.c_size_t(w.numel())


# ----------------------------------------------------------------------------------------------
# Entry points
# ----------------------------------------------------------------------------------------------

def kcs_workspace_bytes(g: Optional[Geometry], n_frames: int, Q: int) -> int:
    gc = g.c() if g is not None else None
    return int(lib().kcs_workspace_bytes(ctypes.byref(gc) if gc is not None else None, n_frames, Q))


def kcs_study_footprint_bytes(g: Geometry, n_frames: int, Q: int) -> int:
    gc = g.c()
    return int(lib().kcs_study_footprint_bytes(ctypes.byref(gc), n_frames, Q))


def alloc_workspace(g: Optional[Geometry], n_frames: int, Q: int, device="cuda"):
    import torch
    return torch.empty(max(kcs_workspace_bytes(g, n_frames, Q), 256), dtype=torch.uint8, device=device)


def kcs_project(g: Geometry, f: Frames, x, q: int, Q: int, ybar, stream=None):
    M = f.M
    gc, fc = g.c(), f.c()
    _check(lib().kcs_project(ctypes.byref(gc), ctypes.byref(fc), _ptr(x, (g.nz, g.ny, g.nx, M), "x"), q, Q,
                             _ptr(ybar, (g.nz, g.subset_size(q, Q), g.n_bin, M), "ybar"), _stream(stream)))


def kcs_backproject(g: Geometry, f: Frames, y, q: int, Q: int, b, sens=None, stream=None):
    M = f.M
    gc, fc = g.c(), f.c()
    _check(lib().kcs_backproject(ctypes.byref(gc), ctypes.byref(fc),
                                 _ptr(y, (g.nz, g.subset_size(q, Q), g.n_bin, M), "y"), q, Q,
                                 _ptr(b, (g.nz, g.ny, g.nx, M), "b"), _ptr(sens, (g.nz, g.ny, g.nx), "sens"),
                                 _stream(stream)))


def kcs_model_tac(f: Frames, k: Kinetics, params, F, J=None, work=None, stream=None):
    n = params.shape[1]
    P = k.n_maps
    fc, kc = f.c(), k.c()
    wp, wn = _work(work)
    _check(lib().kcs_model_tac(ctypes.byref(fc), ctypes.byref(kc), _ptr(params, (P, n), "params"), n,
                               _ptr(F, (n, f.M), "F"), _ptr(J, (n, f.M, P), "J"), wp, wn, _stream(stream)))


def kcs_ki_map(params, ki, stream=None):
    """K_i = K1 k3 / (k2 + k3) per voxel of the maps params [3][...] into ki [...]."""
    n = ki.numel()
    _check(lib().kcs_ki_map(_ptr(params, (3,) + tuple(ki.shape), "params"), n, _ptr(ki, tuple(ki.shape), "ki"),
                            _stream(stream)))


def kcs_rebin_ssrb(n_rings: int, max_ring_diff: int, y3d, y2d, count=None, stream=None):
    """Single-slice rebinning: y3d [2D + 1][R][n_ang][n_bin][M] (span 1, by ring difference and
    first ring) into y2d [2R - 1][n_ang][n_bin][M]; count [2R - 1] (ring pairs per plane) or None."""
    nd, R, n_ang, n_bin, M = tuple(y3d.shape)
    if nd != 2 * max_ring_diff + 1 or R != n_rings:
        raise ValueError("y3d must be [2 * max_ring_diff + 1][n_rings][n_ang][n_bin][M]")
    _check(lib().kcs_rebin_ssrb(n_rings, max_ring_diff, n_ang, n_bin, M, _ptr(y3d, tuple(y3d.shape), "y3d"),
                                _ptr(y2d, (2 * n_rings - 1, n_ang, n_bin, M), "y2d"),
                                _ptr(count, (2 * n_rings - 1,), "count"), _stream(stream)))


def kcs_osl_update(g: Geometry, f: Frames, k: Kinetics, p: Prior, sino, params, q: int, Q: int, x, work,
                   stream=None):
    gc, fc, kc, pc = g.c(), f.c(), k.c(), p.c()
    wp, wn = _work(work)
    _check(lib().kcs_osl_update(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc),
                                _ptr(sino, (g.nz, g.n_ang, g.n_bin, f.M), "sino"),
                                _ptr(params, (k.n_maps, g.nz, g.ny, g.nx), "params"), q, Q,
                                _ptr(x, (g.nz, g.ny, g.nx, f.M), "x"), wp, wn, _stream(stream)))


def kcs_lm_fit(g: Geometry, f: Frames, k: Kinetics, p: Prior, lm: LMOptions, x, params, lam, work, stream=None):
    gc, fc, kc, pc, lc = g.c(), f.c(), k.c(), p.c(), lm.c()
    wp, wn = _work(work)
    _check(lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc), ctypes.byref(lc),
                            _ptr(x, (g.nz, g.ny, g.nx, f.M), "x"), _ptr(params, (k.n_maps, g.nz, g.ny, g.nx), "params"),
                            _ptr(lam, (g.nz, g.ny, g.nx), "lambda"), wp, wn, _stream(stream)))


def kcs_init_state(g: Geometry, f: Frames, sino, xi0, x, params, lam, work, stream=None):
    """xi0: 3 initial map values (K1, k2, k3), or 4 with the blood fraction (params [len(xi0)][...])."""
    gc, fc = g.c(), f.c()
    P = len(xi0)
    xi = (ctypes.c_double * P)(*xi0)
    wp, wn = _work(work)
    _check(lib().kcs_init_state(ctypes.byref(gc), ctypes.byref(fc), _ptr(sino, (g.nz, g.n_ang, g.n_bin, f.M), "sino"),
                                xi, P, _ptr(x, (g.nz, g.ny, g.nx, f.M), "x"),
                                _ptr(params, (P, g.nz, g.ny, g.nx), "params"), _ptr(lam, (g.nz, g.ny, g.nx), "lambda"),
                                wp, wn, _stream(stream)))


def kcs_icm_sweep(g: Geometry, f: Frames, k: Kinetics, p: Prior, lm: LMOptions, sino, Q: int, sweep_idx: int, x,
                  params, lam, work, stream=None):
    gc, fc, kc, pc, lc = g.c(), f.c(), k.c(), p.c(), lm.c()
    wp, wn = _work(work)
    _check(lib().kcs_icm_sweep(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc),
                               ctypes.byref(lc), _ptr(sino, (g.nz, g.n_ang, g.n_bin, f.M), "sino"), Q, sweep_idx,
                               _ptr(x, (g.nz, g.ny, g.nx, f.M), "x"), _ptr(params, (k.n_maps, g.nz, g.ny, g.nx), "params"),
                               _ptr(lam, (g.nz, g.ny, g.nx), "lambda"), wp, wn, _stream(stream)))


def kcs_icm_sweep_noalloc(g: Geometry, f: Frames, k: Kinetics, p: Prior, lm: LMOptions, sino, Q: int,
                          sweep_idx: int, x, params, lam, stream=None):
    """kcs_icm_sweep with the library's static per-GPU scratch as workspace (allocates nothing)."""
    gc, fc, kc, pc, lc = g.c(), f.c(), k.c(), p.c(), lm.c()
    _check(lib().kcs_icm_sweep_noalloc(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc),
                                       ctypes.byref(lc), _ptr(sino, (g.nz, g.n_ang, g.n_bin, f.M), "sino"), Q,
                                       sweep_idx, _ptr(x, (g.nz, g.ny, g.nx, f.M), "x"),
                                       _ptr(params, (k.n_maps, g.nz, g.ny, g.nx), "params"),
                                       _ptr(lam, (g.nz, g.ny, g.nx), "lambda"), _stream(stream)))


@dataclass
class Study:
    """One study of a batched plan: its constants, its sweep range and its device buffers
    (sino (nz, n_ang, n_bin, M), x (nz, ny, nx, M), params (k.n_maps, nz, ny, nx), lam (nz, ny, nx),
    work: uint8 workspace of kcs_workspace_bytes(g, M, Q) bytes)."""
    g: Geometry
    f: Frames
    k: Kinetics
    p: Prior
    lm: LMOptions
    Q: int
    sweep_begin: int
    sweep_end: int
    sino: object
    x: object
    params: object
    lam: object
    work: object

    def c(self) -> c_study:
        g, M = self.g, self.f.M
        wp, wn = _work(self.work)
        return c_study(g.c(), self.f.c(), self.k.c(), self.p.c(), self.lm.c(), self.Q, self.sweep_begin,
                       self.sweep_end, _ptr(self.sino, (g.nz, g.n_ang, g.n_bin, M), "sino"),
                       _ptr(self.x, (g.nz, g.ny, g.nx, M), "x"),
                       _ptr(self.params, (self.k.n_maps, g.nz, g.ny, g.nx), "params"),
                       _ptr(self.lam, (g.nz, g.ny, g.nx), "lambda"), wp, wn)


class Plan:
    """Handle of a kcs_plan; keeps the studies' tensors alive until kcs_plan_destroy."""

    def __init__(self, handle: ctypes.c_void_p, studies):
        self.handle = handle
        self.studies = list(studies)

    def __del__(self):
        kcs_plan_destroy(self)


def kcs_plan_create(studies: Sequence[Study], flags: int = 0, stream=None) -> Plan:
    arr = (c_study * len(studies))(*[s.c() for s in studies])
    h = ctypes.c_void_p()
    _check(lib().kcs_plan_create(arr, len(studies), flags, _stream(stream), ctypes.byref(h)))
    return Plan(h, studies)


def kcs_plan_run(plan: Plan, stream=None):
    if plan.handle is None:
        raise ValueError("plan was destroyed")
    _check(lib().kcs_plan_run(plan.handle, _stream(stream)))


def kcs_plan_describe(plan: Plan) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib().kcs_plan_describe(plan.handle, buf, len(buf)))
    return buf.value.decode()


def kcs_plan_destroy(plan: Plan):
    if plan.handle is not None:
        lib().kcs_plan_destroy(plan.handle)
        plan.handle = None
        plan.studies = []


def kcs_timing_enable(on: bool):
    _check(lib().kcs_timing_enable(1 if on else 0))


def kcs_timing_collect() -> dict:
    """{kind: (total_ms, launches)} for the launches recorded since the last collection."""
    n = len(TIMING_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().kcs_timing_collect(ms, cnt))
    return {k: (ms[i], int(cnt[i])) for i, k in enumerate(TIMING_KINDS)}


def kcs_stream_probe(kind: int, src, dst, groups: int, stream=None):
    """Bandwidth probe: kind 0 reads all of src (uint8/float device tensor) into one partial sum
    per thread in dst (float32, groups * 256); kind 1 copies src into dst (same byte size)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if kind == 0:
        need = groups * 256
        if dst.dtype != torch.float32 or dst.numel() < need:
            raise ValueError(f"dst must hold {need} float32")
    elif dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    for t in (src, dst):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("src and dst must be contiguous device tensors")
    _check(lib().kcs_stream_probe(kind, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                  groups, _stream(stream)))


def kcs_last_error() -> str:
    return lib().kcs_last_error().decode()
