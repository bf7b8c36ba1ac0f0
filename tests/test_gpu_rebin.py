"""Single-slice rebinning on the GPU against the FP64 oracle: bit-exact for integer counts (FP32
sums of integers below 2^24), within FP32 rounding for other values, the ring-pair counts exact,
and entries of ring pairs outside the scanner never read (they hold NaN)."""
import numpy as np
import pytest

import oracle
from kcs_testutil import rel_l2

torch = pytest.importorskip("torch")
from paper_1803_10045_amd import kcs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = "cuda"


def acquisition(R, D, n_ang, n_bin, M, seed, integer=True):
    rng = np.random.default_rng(seed)
    shape = (2 * D + 1, R, n_ang, n_bin, M)
    y = rng.poisson(5.0, shape).astype(np.float32) if integer else rng.random(shape).astype(np.float32)
    for d in range(2 * D + 1):
        for r1 in range(R):
            if not 0 <= r1 + d - D < R:
                y[d, r1] = np.nan
    return y


@pytest.mark.parametrize("R,D,n_ang,n_bin,M", [(1, 0, 3, 5, 1), (5, 2, 7, 9, 3), (16, 15, 60, 64, 24),
                                               (64, 60, 21, 344, 2)])
def test_ssrb_matches_oracle(R, D, n_ang, n_bin, M):
    """Ragged sizes, a single ring, every ring difference, and the mMR's 64 rings (127 planes;
    here 21 of its 252 angles and 2 frames)."""
    y = acquisition(R, D, n_ang, n_bin, M, seed=R + D)
    out = torch.empty((2 * R - 1, n_ang, n_bin, M), device=DEV)
    count = torch.empty(2 * R - 1, device=DEV)
    kcs.kcs_rebin_ssrb(R, D, torch.from_numpy(y).to(DEV), out, count)
    torch.cuda.synchronize()
    ref, cref = oracle.ssrb(y.astype(np.float64), R, D)
    g = out.cpu().numpy()
    print(f"R={R} D={D}: {int(np.isnan(y).sum())} entries outside the scanner; max |diff| {np.abs(g - ref).max():.3g}")
    assert np.array_equal(g.astype(np.float64), ref)
    assert np.array_equal(count.cpu().numpy().astype(np.float64), cref)


def test_ssrb_real_values_and_no_count():
    R, D = 9, 4
    y = acquisition(R, D, 11, 13, 5, seed=3, integer=False)
    out = torch.empty((2 * R - 1, 11, 13, 5), device=DEV)
    kcs.kcs_rebin_ssrb(R, D, torch.from_numpy(y).to(DEV), out)
    torch.cuda.synchronize()
    ref, _ = oracle.ssrb(y.astype(np.float64), R, D)
    e = rel_l2(out.cpu().numpy(), ref)
    print(f"real-valued sinograms: relL2 {e:.2e}")
    assert e < 1e-6
