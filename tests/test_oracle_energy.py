"""Pins of the oracle's energy functional E_p (Section 3.5, eqs.
energyApprox and energyApproxFiner) against values that the mathematics or
the paper fixes, independent of the oracle's own code:

* 2D, unit circle and the 64-point cloud on it: E_2 of the exact circle is
  sqrt(256 (pi/64 - sin(pi/64))) = 7.1035e-2, the paper's reference value for
  its circle test; the discrete E_2 of the circle's signed distance
  approaches it as h -> 0.
* 2D, a straight line y = y0 with constant d = c: the segments tile the
  line, so E_p = c L^(1/p) exactly.
* 2D, one cell crossed on all four edges, worked by hand.
* 3D, a plane z = z0 through the centres of one layer of subcells: exactly
  that layer counts (its neighbours lie h' away, beyond (sqrt 3/2) h'), so
  E_1 with d linear in x is the integral of d over the plane's rectangle
  (the midpoint rule is exact for linear d).  Shifting the plane by 0.2 h'
  brings the next layer within 0.8 h' < (sqrt 3/2) h': two layers count.
* Homogeneity E_p(phi, lam d) = lam E_p(phi, d) and symmetry under phi -> -phi.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth

E2_CIRCLE = math.sqrt(256.0 * (math.pi / 64.0 - math.sin(math.pi / 64.0)))


def circle_case(n):
    g = synth.cube_grid(2, n, -1.5, 1.5)
    X = oracle.node_coords(g)
    phi = (np.linalg.norm(X, axis=1) - 1.0).reshape(g["n"])
    th = 2.0 * np.pi * np.arange(64) / 64.0
    pts = np.stack([np.cos(th), np.sin(th)], 1)
    return g, phi, oracle.distance(pts, g)


@pytest.mark.parametrize("n,tol", [(401, 2e-3), (1601, 5e-4)])
def test_energy_circle_approaches_exact_value(n, tol):
    assert abs(E2_CIRCLE - 7.103510780002126e-02) < 1e-15
    g, phi, d = circle_case(n)
    e2 = oracle.energy(phi, d, g, 2.0)
    assert abs(e2 - E2_CIRCLE) / E2_CIRCLE < tol


@pytest.mark.parametrize("p", [1.0, 2.0, 3.0])
def test_energy_straight_line(p):
    g = synth.cube_grid(2, 41, -1.0, 1.0)
    X = oracle.node_coords(g)
    y0 = 0.1234
    phi = (X[:, 1] - y0).reshape(g["n"])
    c = 0.37
    d = np.full(g["n"], c)
    L = (g["n"][0] - 1) * g["h"]
    assert oracle.energy(phi, d, g, p) == pytest.approx(c * L ** (1.0 / p), rel=1e-13)


def test_energy_four_crossing_cell():
    # vertices (i,j)=3, (i+1,j)=-1, (i,j+1)=-1, (i+1,j+1)=1; centre mean 0.5 lies
    # outside like vertex (i,j): crossings (0.75,0)-(1,0.5) and (0.5,1)-(0,0.75)
    g = {"dim": 2, "n": (2, 2), "lo": (0.0, 0.0), "h": 1.0}
    phi = np.array([[3.0, -1.0], [-1.0, 1.0]])
    d = np.ones((2, 2))
    seg = math.hypot(0.25, 0.5)
    assert oracle.energy(phi, d, g, 1.0) == pytest.approx(2.0 * seg, rel=1e-14)
    # the other pairing would give hypot(0.75, 0.75) + hypot(0.5, 0.5)
    assert abs(2.0 * seg - (math.hypot(0.75, 0.75) + math.hypot(0.5, 0.5))) > 0.5


def plane_case(shift, R=5):
    g = synth.cube_grid(3, 13, -1.0, 1.0)
    h = g["h"]
    hs = h / R
    k0, w0 = 5, 2
    z0 = g["lo"][2] + (k0 + (w0 + 0.5) / R) * h + shift * hs
    X = oracle.node_coords(g)
    phi = (X[:, 2] - z0).reshape(g["n"])
    a, b = 2.0, 0.5
    d = (a + b * X[:, 0]).reshape(g["n"])
    x0, x1 = g["lo"][0], g["lo"][0] + (g["n"][0] - 1) * h
    y0, y1 = g["lo"][1], g["lo"][1] + (g["n"][1] - 1) * h
    integral = (a * (x1 - x0) + 0.5 * b * (x1 ** 2 - x0 ** 2)) * (y1 - y0)
    return g, phi, d, integral


def test_energy_plane_one_layer():
    g, phi, d, integral = plane_case(0.0)
    assert oracle.energy(phi, d, g, 1.0) == pytest.approx(integral, rel=1e-12)


def test_energy_plane_threshold():
    # 0.2 h' off a centre: the next layer's centres are 0.8 h' away (< 0.866 h')
    g, phi, d, integral = plane_case(0.2)
    assert oracle.energy(phi, d, g, 1.0) == pytest.approx(2.0 * integral, rel=1e-12)
    # 0.05 h' off: the neighbours are 0.95 h' and 1.05 h' away
    g, phi, d, integral = plane_case(0.05)
    assert oracle.energy(phi, d, g, 1.0) == pytest.approx(integral, rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_homogeneous_and_symmetric(dim):
    g = synth.cube_grid(dim, 24 if dim == 3 else 64)
    X = oracle.node_coords(g)
    r = np.linalg.norm(X - 0.05, axis=1)
    phi = (r - 0.55 + 0.03 * np.sin(7 * X[:, 0])).reshape(g["n"])
    d = (0.1 + np.abs(np.cos(3 * X[:, 1]))).reshape(g["n"])
    e = oracle.energy(phi, d, g, 2.0)
    assert e > 0
    assert oracle.energy(phi, 3.0 * d, g, 2.0) == pytest.approx(3.0 * e, rel=1e-13)
    assert oracle.energy(-phi, d, g, 2.0) == pytest.approx(e, rel=1e-13)


# ------------------------------------------------ the p = 2 step (Section 2)

def test_p2_with_constant_d_equals_p1_with_half_delta():
    """With d = d0 everywhere and E = d0, C = c (d/E)^(p-1) equals c, and the
    diffusion reach sqrt(C delta d dt / p) at p = 2 is that of p = 1 with
    delta / 2: the two steps agree bit for bit."""
    g = synth.cube_grid(3, 33)
    h = g["h"]
    X = oracle.node_coords(g)
    phi = (np.linalg.norm(X - 0.03, axis=1) - 0.5).reshape(g["n"])
    phi = np.clip(phi, -6 * h, 6 * h)
    d0 = 0.2
    d = np.full(g["n"], d0)
    base = oracle.default_params(3, h)
    p2 = dict(base, p=2.0, energy=d0, delta=1.0)
    p1 = dict(base, p=1.0, delta=0.5)
    a, _, _ = oracle.step(phi, d, g, p2, 0.5 * h, "weno")
    b, _, _ = oracle.step(phi, d, g, p1, 0.5 * h, "weno")
    np.testing.assert_array_equal(a, b)


def test_p2_radial_closed_form():
    """A single cloud point at the origin, phi = |x| - 0.5 near the front:
    at p = 2, C = r / E (d = r, c = 1 inside the cut-off), the drift moves a
    node at radius r to r + C dt and the four foot points lie a distance
    sqrt(2) a off that point across the gradient, a^2 = C delta r dt / 2, so
    phi^{n+1} = sqrt((r + C dt)^2 + C delta r dt) - 0.5 up to interpolation
    error.  Misplacing the factor or the 1/p leaves an O(h) residual."""
    g = synth.cube_grid(3, 65)
    h = g["h"]
    prm = dict(oracle.default_params(3, h), p=2.0, energy=0.4)
    dt = 0.5 * h
    d = oracle.distance_brute(np.zeros((1, 3)), g)
    phi = d - 0.5
    sel = np.nonzero((np.abs(phi.ravel()) <= prm["beta"]) & (d.ravel() > 0.2))[0][:200]
    got, _ = oracle.sl_nodes(phi, d, g, prm, dt, "weno", sel)
    r = d.ravel()[sel]
    E = prm["energy"]

    def closed(C, half):
        return np.sqrt((r + C * dt) ** 2 + (0.5 if half else 1.0) * 2 * C * r * dt) - 0.5

    right = np.abs(got - closed(r / E, True)).max()
    assert right < 0.05 * h
    assert right < 0.1 * np.abs(got - closed(r / E, False)).max()   # 1/p dropped
    assert right < 0.1 * np.abs(got - closed(1.0, True)).max()      # (d/E) dropped
    assert right < 0.1 * np.abs(got - closed(E / r, True)).max()    # inverted ratio


# ------------------------------------------------ stopping test, eq. (deltaEn)

def test_stop_rule_constant_energy_stops_at_the_minimum():
    e = [0.3] * 200
    stops = [n for n in range(200) if oracle.stop_rule(e, n)]
    assert stops[0] == 10


def test_stop_rule_linear_decrease_closed_form():
    """E_2(phi^i) = 1 - a i: consecutive k-means differ by a exactly, so
    Delta_n = a / mean_n, with mean_n = 1 - a (n - (k - 1) / 2)."""
    a = 2e-5
    e = [1.0 - a * i for i in range(120)]
    for n in (10, 30, 60):
        k = min(n, 10)
        mean_n = 1.0 - a * (n - (k - 1) / 2.0)
        delta = a / mean_n
        assert oracle.stop_rule(e, n, tol=delta * (1 + 1e-6))
        assert not oracle.stop_rule(e, n, tol=delta * (1 - 1e-6))


def test_stop_rule_limits():
    e = list(np.linspace(1.0, 0.5, 150))  # Delta about 3e-3 per step: never below 1e-4
    assert not any(oracle.stop_rule(e, n) for n in range(100))
    assert oracle.stop_rule(e, 100)
    assert not oracle.stop_rule([0.2] * 12, 5)  # below the minimum


def test_stop_rule_of_the_library_matches_the_oracle():
    """The C ABI's host-side rule (no device work) against the oracle's."""
    from paper_2410_22205_amd import lsr
    rng = np.random.default_rng(7)
    for trial in range(200):
        n_max = int(rng.integers(1, 130))
        e = list(0.1 + np.cumsum(rng.normal(0.0, 1e-5, n_max + 1)) * rng.choice([0.0, 1.0, 10.0]))
        tol = float(rng.choice([1e-4, 1e-5, 1e-3]))
        for n in range(n_max + 1):
            assert lsr.lsr_energy_stop(e, n, 10, 100, tol) == int(oracle.stop_rule(e, n, tol=tol))
