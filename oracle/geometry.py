"""FP64 oracle: system matrix, ordered subsets, forward and back projection.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline leg of the
benchmark.  The HIP library never imports, links or calls anything in this package.

The system matrix of one plane is built once with Siddon's exact intersection lengths
(``siddon.c``) and stored as a scipy CSR matrix, rows = rays (angle-major), columns = pixels
(row-major y, x).  Direct planes only: every plane uses the same 2D matrix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")


def build_oracle_library(force: bool = False) -> str:
    """Compile ``siddon.c`` and ``kinetics.c`` with gcc into ``liboracle.so`` (seconds)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp,
                               os.path.join(_HERE, "siddon.c"), os.path.join(_HERE, "kinetics.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Geom2D(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double),
                ("n_ang", ctypes.c_int32), ("n_bin", ctypes.c_int32), ("du", ctypes.c_double),
                ("ang0", ctypes.c_double)]


@lru_cache(maxsize=1)
def _lib():
    lib = ctypes.CDLL(build_oracle_library())
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.orc_csr_count.argtypes = [ctypes.POINTER(_Geom2D), i64p]
    lib.orc_csr_count.restype = ctypes.c_int64
    lib.orc_csr_fill.argtypes = [ctypes.POINTER(_Geom2D), i64p, i64p, f64p]
    lib.orc_csr_fill.restype = None
    lib.orc_ray_cos_sin.argtypes = [ctypes.POINTER(_Geom2D), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.orc_siddon_line.argtypes = [ctypes.POINTER(_Geom2D), ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, f64p]
    lib.orc_siddon_line.restype = ctypes.c_int32
    lib.orc_tissue_integrals.argtypes = [ctypes.c_int64, f64p, ctypes.c_int32, f64p, f64p, f64p, ctypes.c_int32,
                                         f64p, f64p, ctypes.c_void_p]
    lib.orc_tissue_integrals.restype = None
    return lib


@dataclass(frozen=True)
class Geometry:
    """Image grid (nx, ny, nz) with square pixels of side ``h`` mm; parallel-beam sinogram of
    ``n_ang`` angles over 180 degrees starting at ``ang0`` and ``n_bin`` bins of ``du`` mm."""
    nx: int
    ny: int
    nz: int
    h: float
    n_ang: int
    n_bin: int
    du: float
    ang0: float = 0.0

    @classmethod
    def from_config(cls, cfg) -> "Geometry":
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.pixel_mm, cfg.n_ang, cfg.n_bin, cfg.bin_mm, cfg.ang0)

    def _c(self) -> _Geom2D:
        return _Geom2D(self.nx, self.ny, self.h, self.n_ang, self.n_bin, self.du, self.ang0)

    @property
    def n_pix(self) -> int:
        return self.nx * self.ny

    def cos_sin(self, a: int):
        c, s = ctypes.c_double(), ctypes.c_double()
        _lib().orc_ray_cos_sin(ctypes.byref(self._c()), int(a), ctypes.byref(c), ctypes.byref(s))
        return c.value, s.value

    def bin_centre(self, b):
        return (np.asarray(b, dtype=np.float64) - 0.5 * (self.n_bin - 1)) * self.du


def siddon_line(geom: Geometry, c: float, s: float, u: float):
    """(pixel indices, lengths) of the line x c + y s = u through the grid of `geom`."""
    lib = _lib()
    g = geom._c()
    work = np.zeros(geom.nx + geom.ny + 4)
    m = lib.orc_siddon_line(ctypes.byref(g), c, s, u, None, None, 0, work)
    idx = np.zeros(max(m, 1), np.int64)
    ln = np.zeros(max(m, 1), np.float64)
    lib.orc_siddon_line(ctypes.byref(g), c, s, u, idx.ctypes.data, ln.ctypes.data, m, work)
    return idx[:m], ln[:m]


_CSR_CACHE: dict = {}


def system_matrix(geom: Geometry) -> sp.csr_matrix:
    """2D system matrix (n_ang*n_bin x nx*ny), FP64 intersection lengths in mm."""
    key = (geom.nx, geom.ny, geom.h, geom.n_ang, geom.n_bin, geom.du, geom.ang0)
    if key in _CSR_CACHE:
        return _CSR_CACHE[key]
    lib = _lib()
    g = geom._c()
    n_rows = geom.n_ang * geom.n_bin
    row_ptr = np.zeros(n_rows + 1, np.int64)
    nnz = lib.orc_csr_count(ctypes.byref(g), row_ptr)
    col = np.zeros(max(nnz, 1), np.int64)
    val = np.zeros(max(nnz, 1), np.float64)
    lib.orc_csr_fill(ctypes.byref(g), row_ptr, col, val)
    A = sp.csr_matrix((val[:nnz], col[:nnz], row_ptr), shape=(n_rows, geom.n_pix))
    if len(_CSR_CACHE) > 4:
        _CSR_CACHE.clear()
    _CSR_CACHE[key] = A
    return A


def subset_angles(n_ang: int, q: int, Q: int) -> np.ndarray:
    """Angles of ordered subset q: every Q-th angle starting at q (interleaved subsets)."""
    return np.arange(q, n_ang, Q)


def subset_rows(geom: Geometry, q: int, Q: int) -> np.ndarray:
    ang = subset_angles(geom.n_ang, q, Q)
    return (ang[:, None] * geom.n_bin + np.arange(geom.n_bin)[None, :]).ravel()


_SUBSET_CACHE: dict = {}


def _subset_matrix(geom: Geometry, q: int, Q: int) -> sp.csr_matrix:
    """Rows of the system matrix that belong to subset q (kept for the geometry's later calls)."""
    key = (geom.nx, geom.ny, geom.h, geom.n_ang, geom.n_bin, geom.du, geom.ang0, q, Q)
    if key not in _SUBSET_CACHE:
        if len(_SUBSET_CACHE) > 256:
            _SUBSET_CACHE.clear()
        _SUBSET_CACHE[key] = system_matrix(geom)[subset_rows(geom, q, Q)]
    return _SUBSET_CACHE[key]


def forward(geom: Geometry, x: np.ndarray, q: int = 0, Q: int = 1) -> np.ndarray:
    """Line integrals sum_v p_vd x_vm for the rays of subset q.

    x: (nz, ny, nx, M) -> (nz, A_q, n_bin, M)."""
    nz, M = x.shape[0], x.shape[-1]
    P = _subset_matrix(geom, q, Q)
    X = np.ascontiguousarray(np.moveaxis(x.reshape(nz, geom.n_pix, M), 1, 0)).reshape(geom.n_pix, nz * M)
    Y = P @ X  # (rays_q, nz*M)
    A_q = len(subset_angles(geom.n_ang, q, Q))
    return np.ascontiguousarray(np.moveaxis(Y.reshape(A_q * geom.n_bin, nz, M), 1, 0)).reshape(nz, A_q, geom.n_bin, M)


def back(geom: Geometry, y: np.ndarray, q: int = 0, Q: int = 1) -> np.ndarray:
    """Adjoint of :func:`forward`: sum_{d in S_q} p_vd y_dm.  y: (nz, A_q, n_bin, M) -> (nz, ny, nx, M)."""
    nz, M = y.shape[0], y.shape[-1]
    P = _subset_matrix(geom, q, Q)
    Y = np.ascontiguousarray(np.moveaxis(y.reshape(nz, -1, M), 1, 0)).reshape(-1, nz * M)
    X = P.T @ Y  # (n_pix, nz*M)
    return np.ascontiguousarray(np.moveaxis(X.reshape(geom.n_pix, nz, M), 1, 0)).reshape(nz, geom.ny, geom.nx, M)


def subset_sensitivity(geom: Geometry, q: int = 0, Q: int = 1) -> np.ndarray:
    """sum_{d in S_q} p_vd per pixel, (ny, nx)."""
    P = _subset_matrix(geom, q, Q)
    return np.asarray(P.sum(axis=0)).reshape(geom.ny, geom.nx)
