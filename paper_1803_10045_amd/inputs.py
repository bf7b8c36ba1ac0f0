"""Seeded synthetic inputs for dynamic FDG PET studies.

This module only *describes* studies: grid and sinogram shapes, the frame
schedule, the plasma input parameters, the true kinetic-parameter maps of a
phantom, prior hyper-parameters derived from the phantom, and a seeded Poisson
sampler.  It holds none of the reconstruction or kinetic-model arithmetic: a
caller turns the true maps into activity and expected counts with its own model
and projector (the FP64 oracle in the tests, the HIP library in the benchmark),
then draws the measured counts with :func:`poisson_counts`.

Everything is drawn from ``numpy.random.Generator(PCG64(seed))`` so both sides
see identical inputs for the same seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

# Frame schedule: 24 frames over 40 min, (count, seconds) per block.
FRAME_BLOCKS: Tuple[Tuple[int, float], ...] = ((6, 10.0), (6, 30.0), (4, 60.0), (4, 180.0), (4, 300.0))
# Schedule printed with the simulation (Eq. 8).  Its blocks add up to 2340 s,
# not the 40 min the text states; kept as a preset only.
FRAME_BLOCKS_EQ8: Tuple[Tuple[int, float], ...] = ((12, 10.0), (2, 30.0), (4, 60.0), (1, 120.0), (4, 300.0), (1, 600.0))

# Feng plasma input  Cp(t) = (A1 t - A2 - A3) e^{l1 t} + A2 e^{l2 t} + A3 e^{l3 t},  t in minutes.
FENG = dict(A1=851.1, A2=21.88, A3=20.81, l1=-4.134, l2=-0.1191, l3=-0.01043)
VB = 0.05  # fixed blood fraction of the irreversible two-tissue model

# (K1 [ml/g/min], k2 [1/min], k3 [1/min]) of the tissue classes.
WHITE = (0.054, 0.109, 0.045)
GRAY = (0.102, 0.130, 0.062)
HOT = (0.12, 0.10, 0.12)

# Initial kinetic parameters, damping and box bounds of the per-voxel fit.
XI0 = (0.08, 0.12, 0.05)
LM_TAU = 1e-3
LM_LAM_MIN, LM_LAM_MAX = 1e-8, 1e8
LM_LO = (0.0, 1e-4, 0.0)
LM_HI = (2.0, 2.0, 1.0)
# With the blood fraction fitted as a fourth map: its initial value and box.
XI0_VB = VB
LM_LO_VB, LM_HI_VB = 0.0, 1.0
# A step is kept only if it lowers the voxel objective by more than this fraction of its value:
# the fit of a voxel counts as converged to this relative tolerance of its objective, and a
# step that gains less is treated as no progress (rejected, damping raised).
LM_ETA = 1e-3
BETA_KP = 0.1


def frame_times(blocks=FRAME_BLOCKS) -> Tuple[np.ndarray, np.ndarray]:
    """Frame start and end times in minutes (FP64), contiguous from t=0."""
    durs = np.concatenate([np.full(n, s / 60.0) for n, s in blocks])
    t1 = np.cumsum(durs)
    t0 = np.concatenate([[0.0], t1[:-1]])  # each frame starts exactly where the previous one ends
    return t0, t1


@dataclass
class StudyConfig:
    name: str
    nx: int
    ny: int
    nz: int
    pixel_mm: float
    plane_mm: float
    n_ang: int
    n_bin: int
    bin_mm: float
    counts: float  # expected true coincidences over the scan
    bg_frac: float  # flat background, as a fraction of `counts`
    Q: int  # ordered subsets per OSL pass
    n_sweeps: int
    n_lm: int = 5
    beta_h: float = 0.1
    phantom: str = "brain"  # "disk" (single-slice) or "brain" (ellipsoid with lesions)
    n_lesions: int = 6
    seed: int = 1
    ang0: float = 0.0
    frame_blocks: Tuple[Tuple[int, float], ...] = FRAME_BLOCKS  # (count, seconds) per block

    @property
    def n_frames(self) -> int:
        return sum(n for n, _ in self.frame_blocks)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz


def disk64() -> StudyConfig:
    """64x64 single slice, 4 mm pixels, 60 angles x 64 bins, 2e6 counts + 10 % background."""
    return StudyConfig("disk_64x64x1", 64, 64, 1, 4.0, 4.0, 60, 64, 4.0, 2e6, 0.10, Q=4, n_sweeps=10,
                       phantom="disk", n_lesions=3, seed=1)


def brain128() -> StudyConfig:
    """128x128x47 direct planes at 2.5 mm, 168 angles x 128 bins, 5e7 counts + 10 %."""
    return StudyConfig("brain_128x128x47", 128, 128, 47, 2.5, 2.5, 168, 128, 2.5, 5e7, 0.10, Q=6, n_sweeps=20,
                       phantom="brain", n_lesions=6, seed=1)


def brain344() -> StudyConfig:
    """Clinical-scale 344x344x127 (2.09 x 2.09 x 2.03 mm), 252 angles x 344 bins, 3e8 counts + 15 %."""
    return StudyConfig("brain_344x344x127", 344, 344, 127, 2.09, 2.03, 252, 344, 2.09, 3e8, 0.15, Q=21, n_sweeps=10,
                       phantom="brain", n_lesions=12, seed=1)


CONFIGS = {"disk64": disk64, "brain128": brain128, "brain344": brain344}


def batch_configs(n_studies: int = 32, seed: int = 4) -> List[StudyConfig]:
    """Uneven batch: slice counts uniform in 8..127, matrix 128 or 172 (p=1/2),
    bins = matrix, angles = round(1.3 matrix), 4e5 counts per slice, 6 subsets, 10 sweeps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_studies):
        nz = int(rng.integers(8, 128))
        n = 128 if rng.random() < 0.5 else 172
        pix = 2.5 if n == 128 else 4.18
        n_ang = int(round(1.3 * n))
        out.append(StudyConfig(f"batch{i:02d}_{n}x{n}x{nz}", n, n, nz, pix, 2.5, n_ang, n, pix, 4e5 * nz, 0.10,
                               Q=6, n_sweeps=10, phantom="brain", n_lesions=6, seed=1000 + i))
    return out


SERVE_SIZES = (
    # (matrix, planes, angles, pixel mm, subsets, sweeps, counts, bg fraction), probability
    ((64, 1, 60, 4.0, 4, 10, 2e6, 0.10), 0.4),
    ((128, 47, 168, 2.5, 6, 20, 5e7, 0.10), 0.3),
    ((172, 64, 224, 4.18, 6, 10, 4e5 * 64, 0.10), 0.2),
    ((344, 127, 252, 2.09, 21, 10, 3e8, 0.15), 0.1),
)


def request_stream(n_requests: int = 200, rate_hz: float = 4.0, seed: int = 7,
                   sizes=SERVE_SIZES) -> List[Tuple[float, StudyConfig]]:
    """Poisson arrivals (exponential gaps at `rate_hz`) with sizes drawn from `sizes`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = np.array([p for _, p in sizes])
    t = 0.0
    out = []
    for j in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        k = int(rng.choice(len(sizes), p=probs / probs.sum()))
        (n, nz, n_ang, pix, Q, sweeps, counts, bg), _ = sizes[k]
        cfg = StudyConfig(f"req{j:03d}_{n}x{n}x{nz}", n, n, nz, pix, 2.5, n_ang, n, pix, counts, bg, Q=Q,
                          n_sweeps=sweeps, phantom="disk" if nz == 1 else "brain",
                          n_lesions=3 if nz == 1 else (12 if n == 344 else 6), seed=5000 + j)
        out.append((t, cfg))
    return out


def scaled(cfg: StudyConfig, **kw) -> StudyConfig:
    """Copy of `cfg` with fields replaced (e.g. fewer planes for a quick test)."""
    return replace(cfg, **kw)


# ----------------------------------------------------------------------------------------------
# Phantoms
# ----------------------------------------------------------------------------------------------

def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


# (K1, k2, k3) of the three tissue regions of the simulation table (Sec. III-A, Table I); its
# blood region has no tissue (K1 = 0) and carries the plasma input itself.
TABLE1_INNER = (0.75, 0.35, 0.031)
TABLE1_MIDDLE = (0.62, 0.30, 0.026)
TABLE1_OUTER = (0.51, 0.27, 0.018)
RING_REGIONS = {1: "blood", 2: "inner", 3: "middle", 4: "outer"}


def ring_labels(cfg: StudyConfig) -> np.ndarray:
    """Stand-in for the simulation phantom (its figure is not available): per voxel 0 outside,
    1 in a central blood square of half-side 0.06 n, and 2 / 3 / 4 in concentric rings (inner,
    middle, outer) out to radii 0.18 n, 0.30 n and 0.42 n, n the matrix size; every plane alike."""
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    n = float(min(nx, ny))
    y = _centres(ny)[:, None]
    x = _centres(nx)[None, :]
    r = np.sqrt(x * x + y * y)
    lab = np.zeros((ny, nx), dtype=np.int32)
    lab[r <= 0.42 * n] = 4
    lab[r <= 0.30 * n] = 3
    lab[r <= 0.18 * n] = 2
    lab[(np.abs(x) <= 0.06 * n) & (np.abs(y) <= 0.06 * n)] = 1
    return np.broadcast_to(lab, (nz, ny, nx)).copy()


def rings_config(n: int = 128, nz: int = 4, counts_per_plane: float = 4e6, seed: int = 41) -> StudyConfig:
    """The comparison study: the ring phantom on an n x n grid (256 mm field), 1.3 n angles,
    n bins, 6 subsets, 10 sweeps, the simulation's frame blocks (FRAME_BLOCKS_EQ8).  Its blood
    square carries the plasma input itself: its activity is the frame average of Cp."""
    h = 256.0 / n
    return StudyConfig(f"rings_{n}x{n}x{nz}", n, n, nz, h, h, int(round(1.3 * n)), n, h, counts_per_plane * nz,
                       0.1, Q=6, n_sweeps=10, phantom="rings", n_lesions=0, seed=seed, frame_blocks=FRAME_BLOCKS_EQ8)


def phantom_maps(cfg: StudyConfig) -> Tuple[np.ndarray, np.ndarray]:
    """True kinetic maps ``(3, nz, ny, nx)`` FP64 (K1, k2, k3) and the object mask ``(nz, ny, nx)``.

    Outside the object all three maps are 0 and the object carries no activity.
    "disk": white-matter disk of radius 24 px, a gray-matter rim out to 28 px and three hot
    disks of radius 3 px centred 12 px from the centre at 0, 120 and 240 degrees (scaled with
    the matrix for grids other than 64).  "brain": ellipsoid with semi-axes (0.36 nx, 0.44 ny,
    0.45 nz), a gray-matter shell 4 voxels thick at 128 (scaled with the matrix), white-matter
    core, and lesions of radius U[3, 6] voxels (scaled) centred in the core, each parameter
    drawn U[0.7, 1.3] x gray matter.  Voxels are assigned by their centres.
    """
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    z = _centres(nz)[:, None, None]
    y = _centres(ny)[None, :, None]
    x = _centres(nx)[None, None, :]
    maps = np.zeros((3, nz, ny, nx))
    if cfg.phantom == "disk":
        s = nx / 64.0
        r = np.sqrt(x * x + y * y) * np.ones((nz, 1, 1))
        obj = r <= 28 * s
        wm = r <= 24 * s
        for p in range(3):
            maps[p][obj] = GRAY[p]
            maps[p][wm] = WHITE[p]
        for k in range(3):
            phi = 2 * np.pi * k / 3
            cx, cy = 12 * s * np.cos(phi), 12 * s * np.sin(phi)
            hot = (x - cx) ** 2 + (y - cy) ** 2 <= (3 * s) ** 2
            hot = hot * np.ones((nz, 1, 1), dtype=bool)
            for p in range(3):
                maps[p][hot] = HOT[p]
        return maps, obj
    if cfg.phantom == "rings":
        labels = ring_labels(cfg)
        # blood square: K1 = 0 (no tissue), its k2, k3 (which then do not change the model TAC)
        # set to the fit's start so that the model stays defined (k2 + k3 > 0)
        for reg, par in ((1, (0.0, XI0[1], XI0[2])), (2, TABLE1_INNER), (3, TABLE1_MIDDLE), (4, TABLE1_OUTER)):
            for p in range(3):
                maps[p][labels == reg] = par[p]
        return maps, labels > 0
    if cfg.phantom != "brain":
        raise ValueError(cfg.phantom)
    s = nx / 128.0
    ax, ay, az = 0.36 * nx, 0.44 * ny, max(0.45 * nz, 0.5)
    rho = (x / ax) ** 2 + (y / ay) ** 2 + (z / az) ** 2
    obj = rho <= 1.0
    th = 4.0 * s
    bx, by, bz = ax - th, ay - th, az - th
    if bz > 0:
        core = (x / bx) ** 2 + (y / by) ** 2 + (z / bz) ** 2 <= 1.0
    else:
        core = np.zeros_like(obj)
    for p in range(3):
        maps[p][obj] = GRAY[p]
        maps[p][core] = WHITE[p]
    for _ in range(cfg.n_lesions):
        rad = rng.uniform(3.0, 6.0) * s
        par = [GRAY[p] * rng.uniform(0.7, 1.3) for p in range(3)]
        if bz > 0:
            while True:  # centre uniform in the white-matter core
                c = rng.uniform(-1.0, 1.0, 3)
                if (c * c).sum() <= 1.0:
                    break
            cx, cy, cz = c[0] * bx, c[1] * by, c[2] * bz
        else:
            while True:
                c = rng.uniform(-1.0, 1.0, 3)
                if (c * c).sum() <= 1.0:
                    break
            cx, cy, cz = c[0] * ax * 0.7, c[1] * ay * 0.7, c[2] * az
        les = ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= rad * rad) & obj
        for p in range(3):
            maps[p][les] = par[p]
    return maps, obj


def huber_delta(maps: np.ndarray, mask: np.ndarray) -> float:
    """Huber threshold: 0.01 x the mean true K1 over object voxels (same for all three maps)."""
    return 0.01 * float(maps[0][mask].mean())


def poisson_counts(expected: np.ndarray, seed: int) -> np.ndarray:
    """Poisson draws of an expected-count array, returned as FP32 (exact integers)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5151])))
    return rng.poisson(np.asarray(expected, dtype=np.float64)).astype(np.float32)


MU_WATER_PER_MM = 0.0096  # linear attenuation of water at 511 keV


def correction_sinogram(nz: int, n_ang: int, n_bin: int, bin_mm: float, radius_mm: float, seed: int = 21,
                        dead_bins: int = 2) -> np.ndarray:
    """Multiplicative correction per ray, (nz, n_ang, n_bin) float32: the attenuation of a water
    cylinder of the given radius centred in the field (exp(-mu L), L the chord of the ray through
    it) times detector-pair efficiencies drawn uniformly in [0.8, 1.2], with `dead_bins` radial
    bins of zero efficiency (a detector gap) at one angle of every plane."""
    rng = np.random.default_rng(seed)
    u = (np.arange(n_bin) - 0.5 * (n_bin - 1)) * bin_mm
    chord = 2.0 * np.sqrt(np.maximum(radius_mm ** 2 - u ** 2, 0.0))
    att = np.exp(-MU_WATER_PER_MM * chord)
    eff = rng.uniform(0.8, 1.2, (nz, n_ang, n_bin))
    mult = att[None, None, :] * eff
    if dead_bins > 0:
        mult[:, n_ang // 3, n_bin // 2:n_bin // 2 + dead_bins] = 0.0
    return mult.astype(np.float32)
