"""Pins of the oracle's cloud resolution h_S (Section 4, the text after
eq. dxdt): the paper's printed value for its 64-point circle, brute force
over all pairs on small clouds, duplicates and a regular lattice."""
import itertools
import math

import numpy as np
import pytest

import oracle
from conftest import read_golden_values


def test_circle_of_64_points_as_printed():
    gold = read_golden_values("cloud_spacing.txt")["circle64_h_S"]
    th = 2.0 * np.pi * np.arange(64) / 64.0
    pts = np.stack([np.cos(th), np.sin(th)], 1)
    sample = np.random.default_rng(3).choice(64, size=6, replace=False)  # 10 %
    h = oracle.cloud_spacing(pts, sample)
    assert abs(h - gold) < 5e-5                       # the printed 3 digits
    assert abs(h - 2.0 * math.sin(math.pi / 64.0)) < 1e-15  # the chord


@pytest.mark.parametrize("dim", [2, 3])
def test_brute_force_small_cloud(dim):
    rng = np.random.default_rng(10 + dim)
    pts = rng.random((40, dim))
    sample = [0, 7, 13, 39]
    want = []
    for s in sample:
        best = math.inf
        for q in range(len(pts)):
            if q == s:
                continue
            best = min(best, math.sqrt(sum((pts[s][a] - pts[q][a]) ** 2 for a in range(dim))))
        want.append(best)
    assert oracle.cloud_spacing(pts, sample) == pytest.approx(sum(want) / len(want), rel=1e-14)


def test_duplicates_and_lattice():
    a = 0.125
    pts = np.array(list(itertools.product(range(5), range(4), range(3))), dtype=np.float64) * a
    assert oracle.cloud_spacing(pts, range(len(pts))) == pytest.approx(a, rel=1e-15)
    dup = np.vstack([pts, pts[:1]])  # point 0 twice: its neighbour is at distance 0
    assert oracle.cloud_spacing(dup, [0]) == 0.0
