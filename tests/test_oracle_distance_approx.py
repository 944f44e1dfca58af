"""Pins of the oracle's approximate distance field (Section 3.4): exact at
the nodes of a 4^dim box around each cloud point, fast sweeping elsewhere.

* One interior point fixes exactly 4^dim nodes, the box of the reading.
* A line of points lying on every grid row at x = c: the exact distance is
  |x - c| and the sweep, exact for data varying along one axis, reproduces
  it everywhere.
* On scattered and surface clouds the first-order sweep stays within 1.5h
  of the exact field, and the boxed nodes keep the exact values.
"""
import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth


@pytest.mark.parametrize("dim", [2, 3])
def test_one_point_fixes_a_box_of_4_nodes_per_axis(dim):
    g = synth.cube_grid(dim, 21)
    _, fixed, _ = oracle.distance_approx(np.array([[0.013, -0.07, 0.041][:dim]]), g)
    assert int(fixed.sum()) == 4 ** dim


@pytest.mark.parametrize("dim", [2, 3])
def test_line_of_points_is_reproduced(dim):
    g = synth.cube_grid(dim, 33 if dim == 2 else 17)
    h = g["h"]
    c = 0.031
    rows = oracle.node_coords(g)[:, 1:]
    rows = np.unique(rows, axis=0)
    pts = np.hstack([np.full((len(rows), 1), c), rows])
    d, _, _ = oracle.distance_approx(pts, g)
    X = oracle.node_coords(g)
    np.testing.assert_allclose(d.ravel(), np.abs(X[:, 0] - c), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["scattered", "surface"])
def test_first_order_error(dim, kind):
    g = synth.cube_grid(dim, 101 if dim == 2 else 41)
    h = g["h"]
    if kind == "scattered":
        pts = np.random.default_rng(5).uniform(-0.6, 0.6, (20, dim))
    elif dim == 3:
        pts = synth.torus_cloud(3000, 0.5, 0.2, 0.0, seed=3)
    else:
        pts = synth.circle_cloud(300, 0.5, seed=3)
    d, fixed, _ = oracle.distance_approx(pts, g)
    exact = oracle.distance(pts, g)
    np.testing.assert_array_equal(d[fixed == 1], exact[fixed == 1])
    assert np.abs(d - exact).max() <= 1.5 * h
