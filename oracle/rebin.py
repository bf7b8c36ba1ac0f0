"""FP64 oracle: single-slice rebinning of a 3D acquisition into direct and cross planes.

TEST INFRASTRUCTURE ONLY (see geometry.py).  The human study of Sec. IV was recorded as 3D
listmode data and rebinned into the sinograms a direct-plane reconstruction takes.  A scanner of
R rings records one sinogram per ring pair (r1, r2); the lines of response of that pair cross the
axis half way between the two rings, on plane r1 + r2 of the 2R - 1 planes spaced half a ring
apart, and single-slice rebinning assigns the whole sinogram to that plane.
"""
from __future__ import annotations

import numpy as np


def ssrb(y3d: np.ndarray, n_rings: int, max_ring_diff: int):
    """y3d: [2D + 1][R][n_ang][n_bin][M], the sinogram of ring pair (r1, r1 + delta) at
    [delta + D][r1].  Returns the rebinned planes [2R - 1][n_ang][n_bin][M] (FP64) and the number
    of ring pairs that each plane received."""
    R, D = n_rings, max_ring_diff
    y3d = np.asarray(y3d)
    out = np.zeros((2 * R - 1,) + y3d.shape[2:])
    count = np.zeros(2 * R - 1)
    for r1 in range(R):
        for r2 in range(R):
            if abs(r2 - r1) > D:
                continue
            out[r1 + r2] += y3d[r2 - r1 + D, r1]
            count[r1 + r2] += 1
    return out, count
