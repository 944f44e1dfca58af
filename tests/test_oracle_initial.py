"""Pins of the oracle's initial data from the cloud (Section 3.6): external
marking from the grid's boundary, d - gamma_S there, fast sweeping of the
first-order upwind eikonal discretisation inside, sign reversed inside.

* A plane: the internal values are the one-dimensional upwind chain from
  the nearest external node, u = (d_e - gamma_S) + |x - x_e| (the scheme is
  exact for data that vary along one axis).
* One cloud point: phi0 is the signed distance of the ball of radius gamma_S
  within 2h (the first-order scheme, started from external values up to h
  outside the ball).
* A closed shell of points with h_S ~ h and gamma_S = 2 h_S (the paper's
  first run): outside is external, the centre is not, and deep inside
  phi0 = |x| - (r + gamma_S) within 1.5h.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth


@pytest.mark.parametrize("dim", [2, 3])
def test_plane_gives_the_upwind_chain(dim):
    g = synth.cube_grid(dim, 41 if dim == 2 else 21)
    h = g["h"]
    X = oracle.node_coords(g)
    d = np.abs(X[:, 0] - 0.03).reshape(g["n"])
    gs = 0.2
    phi, ext, cycles = oracle.phi0_from_cloud(d, g, gs)
    np.testing.assert_array_equal(ext, (d >= gs).astype(np.uint8))
    x = g["lo"][0] + h * np.arange(g["n"][0])
    dx = np.abs(x - 0.03)
    e = np.nonzero(dx >= gs)[0]
    want = np.empty(len(x))
    for i in range(len(x)):
        want[i] = dx[i] - gs if dx[i] >= gs else -min(dx[k] - gs + abs(i - k) * h for k in e)
    full = np.broadcast_to(want.reshape((-1,) + (1,) * (dim - 1)), g["n"])
    np.testing.assert_allclose(phi, full, rtol=0, atol=1e-12)
    assert cycles < 10


@pytest.mark.parametrize("dim", [2, 3])
def test_one_point_gives_the_ball(dim):
    g = synth.cube_grid(dim, 81 if dim == 2 else 41)
    h = g["h"]
    X = oracle.node_coords(g)
    d = np.linalg.norm(X - np.array([0.05, -0.02, 0.01][:dim]), axis=1).reshape(g["n"])
    gs = 0.3
    phi, ext, _ = oracle.phi0_from_cloud(d, g, gs)
    np.testing.assert_array_equal(ext, (d >= gs).astype(np.uint8))
    np.testing.assert_array_equal(phi[ext == 1], (d - gs)[ext == 1])
    inside = ext == 0
    assert (phi[inside] < 0).all()
    assert np.abs(phi - (d - gs))[inside].max() <= 2.0 * h


def _shell(dim, g, r):
    h = g["h"]
    if dim == 2:
        n = int(round(2 * math.pi * r / h))
        t = 2 * np.pi * np.arange(n) / n
        return np.stack([r * np.cos(t), r * np.sin(t)], 1)
    n = int(round(4 * math.pi * r * r / (h * h)))  # golden spiral, spacing ~ h
    k = np.arange(n) + 0.5
    z = 1 - 2 * k / n
    t = math.pi * (1 + 5 ** 0.5) * k
    s = np.sqrt(1 - z * z)
    return r * np.stack([s * np.cos(t), s * np.sin(t), z], 1)


@pytest.mark.parametrize("dim", [2, 3])
def test_closed_shell(dim):
    g = synth.cube_grid(dim, 81 if dim == 2 else 41)
    h = g["h"]
    r = 0.5
    pts = _shell(dim, g, r)
    d = oracle.distance(pts, g)
    hs = oracle.cloud_spacing(pts, np.arange(0, len(pts), 10))
    assert 0.9 * h < hs < 1.1 * h
    gs = 2 * hs
    phi, ext, _ = oracle.phi0_from_cloud(d, g, gs)
    X = oracle.node_coords(g)
    rr = np.linalg.norm(X, axis=1).reshape(g["n"])
    assert ext[rr > r + gs + 2 * h].all()
    assert ext.ravel()[np.argmin(rr)] == 0
    assert (phi[ext == 0] < 0).all() and (phi[ext == 1] >= 0).all()
    deep = (ext == 0) & (rr < r - gs)
    assert deep.sum() > 50
    assert np.abs(phi - (rr - (r + gs)))[deep].max() <= 1.5 * h
