"""The comparison study's inputs against the values the paper prints (tests/golden: Table I and
the frame blocks of Eq. 8, Sec. III-A)."""
import json
import os

import numpy as np

from paper_1803_10045_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "simulation_setup.json")


def test_table_1_parameters():
    g = json.load(open(GOLDEN))["table_1"]
    assert tuple(g["inner"]) == inputs.TABLE1_INNER
    assert tuple(g["middle"]) == inputs.TABLE1_MIDDLE
    assert tuple(g["outer"]) == inputs.TABLE1_OUTER
    assert g["blood"][0] == 0.0  # no tissue in the blood region (its K1 is 0)


def test_eq8_frame_blocks():
    g = json.load(open(GOLDEN))["eq_8_frame_blocks"]
    assert [list(map(float, b)) for b in g["blocks"]] == [[float(n), float(s)] for n, s in inputs.FRAME_BLOCKS_EQ8]
    t0, t1 = inputs.frame_times(inputs.FRAME_BLOCKS_EQ8)
    assert len(t0) == g["frames"] == 24
    assert t1[-1] * 60.0 == sum(n * s for n, s in g["blocks"]) == 2340.0  # 39 min, not the 40 the text states
    assert np.all(t0[1:] == t1[:-1]) and t0[0] == 0.0
