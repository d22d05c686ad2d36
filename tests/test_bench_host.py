"""Host-side helpers of bench.py: strict-JSON output, the comment-blind
source hash that keys the counter records, and the lane-node counts the
roofline figures divide by."""
import math

import pytest

import bench


def test_no_nan_makes_strict_json():
    import json
    x = {"a": float("nan"), "b": [1.0, float("inf"), {"c": -float("inf")}], "d": 2}
    y = bench._no_nan(x)
    assert y == {"a": None, "b": [1.0, None, {"c": None}], "d": 2}
    json.dumps(y, allow_nan=False)


def test_source_code_ignores_comments_and_layout():
    a = "int f(int x) {  // one\n  return x + 1; /* two\n three */ }\n"
    b = "int f(int x) {\n return x + 1; }  // different comment\n"
    c = "int f(int x) { return x + 2; }"
    assert bench.source_code(a) == bench.source_code(b)
    assert bench.source_code(a) != bench.source_code(c)


@pytest.mark.parametrize("P,K,W", [(8, 40, 4), (8, 32, 4), (4, 24, 4), (2, 16, 4)])
def test_lattice_lane_nodes(P, K, W):
    span = P * (62 * W + 2)
    out = span - 4 * K
    for L in (3, 100, out - 1, out, out + 1, 3 * out + 7, 20000):
        c = bench.lattice_lane_nodes(L, P, K, W)
        # whole wavefronts of 64 P lane-nodes, at least the lattice plus
        # the halos of each of its tiles, at most full tiles
        tiles = math.ceil(L / out)
        assert c % (64 * P) == 0
        assert c >= L
        assert c <= tiles * 64 * P * W


def test_batch_computed_resident_wavefronts():
    import numpy as np
    lens = np.array([16, 496, 497, 5952, 9000])
    res = np.array([True, True, True, True, False])
    c = bench.batch_computed(lens, res, 8, 40, 4)
    want = 512 * (1 + 1 + 2 + 12) + bench.lattice_lane_nodes(9000, 8, 40, 4)
    assert c == want
