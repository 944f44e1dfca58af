"""Pins of the oracle's semi-Lagrangian step (Section 3.1 with the cut and
cut-off of Section 3.8), its distance field (Section 2) and its initial data,
against closed forms, exact translations, symmetry and brute force."""
import math

import numpy as np
import pytest

import oracle
from conftest import read_golden_values

RNG = np.random.default_rng(99)


def _grid(dim, n, lo=-1.0, hi=1.0):
    return {"dim": dim, "n": (n,) * dim, "lo": (lo,) * dim, "h": (hi - lo) / (n - 1)}


def test_paper_constants_are_the_defaults():
    gold = read_golden_values("paper_constants.txt")
    for dim in (2, 3):
        h = 0.1
        p = oracle.default_params(dim, h)
        assert p["grad_C"] == gold["grad_C"] and p["grad_alpha"] == gold["grad_alpha"]
        assert p["gamma"] == pytest.approx(gold[f"band_gamma_{dim}d"] * h)
        assert p["beta"] == pytest.approx(gold[f"cutoff_beta_{dim}d"] * h)
    # eps = dx^2: with both indicators zero the weights are the linear ones,
    # and the ratio alpha_L/alpha_R = (C_L/C_R) * ((I_R+eps)/(I_L+eps))^2 fixes eps.
    dx = 0.37
    v = np.array([0.0, 0.0, 0.0, 1.0])  # I_L = 0, I_R = 1/dx^2
    _, parts = oracle.weno1d(v, 0.5, dx, parts=True)
    eps = gold["weno_eps_over_dx2"] * dx * dx
    ratio = (parts["CL"] / parts["CR"]) * ((parts["IR"] + eps) / (parts["IL"] + eps)) ** 2
    assert parts["wL"] / parts["wR"] == pytest.approx(ratio, rel=1e-12)


def test_cutoff_shape():
    beta, gamma = 3.0, 6.0
    assert oracle.cutoff(beta, beta, gamma) == 1.0
    assert oracle.cutoff(gamma, beta, gamma) == pytest.approx(0.0, abs=1e-15)
    assert oracle.cutoff(0.0, beta, gamma) == 1.0
    assert oracle.cutoff(7.0, beta, gamma) == 0.0
    e = 1e-6
    for x in (beta, gamma):
        slope = (oracle.cutoff(x + e, beta, gamma) - oracle.cutoff(x - e, beta, gamma)) / (2 * e)
        assert abs(slope) < 1e-5  # C^1 joins
    xs = np.linspace(beta, gamma, 50)
    cs = [oracle.cutoff(x, beta, gamma) for x in xs]
    assert all(a >= b for a, b in zip(cs, cs[1:]))
    for x in xs:
        assert oracle.cutoff(-x, beta, gamma) == oracle.cutoff(x, beta, gamma)


def _params(dim, h, **kw):
    return oracle.default_params(dim, h, **kw)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["q1", "weno"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_translation_by_whole_cells_is_exact(dim, kind, axis):
    """delta = 0, d = x_axis + 1 (so grad d = e_axis), c = 1 everywhere and
    C dt = k h: the update must be phi(x_j + k h e_axis), a whole-cell shift."""
    if axis >= dim:
        pytest.skip("2D grid")
    n, k = 11, 2
    g = _grid(dim, n)
    h = g["h"]
    X = oracle.node_coords(g)
    phi = (0.3 * X[:, 0] - 0.2 * X[:, 1] + 0.1 * np.sin(2 * X[:, -1]) + 0.05 * X[:, 0] * X[:, -1])
    phi = phi.reshape(g["n"])
    d = (X[:, axis] + 1.0).reshape(g["n"])
    prm = _params(dim, h, delta=0.0, gamma=50.0, beta=40.0)
    out, band, _ = oracle.step(phi, d, g, prm, k * h, kind)
    assert band.all()
    src = [slice(None)] * dim
    dst = [slice(None)] * dim
    src[axis] = slice(k, None)
    dst[axis] = slice(0, n - k)
    want = phi[tuple(src)]
    got = out[tuple(dst)]
    # nodes off the domain boundary: there the centred difference of the
    # linear d is exactly e_axis (one-sided differences elsewhere)
    sel = [slice(1, -1)] * dim
    sel[axis] = slice(1, None)
    np.testing.assert_allclose(got[tuple(sel)], want[tuple(sel)], atol=1e-13)


@pytest.mark.parametrize("dim,kind,min_ratio", [(2, "q1", 3.0), (3, "q1", 3.0),
                                                (2, "weno", 6.0), (3, "weno", 6.0)])
def test_one_step_radial_closed_form(dim, kind, min_ratio):
    """Cloud = {0}, so d = |x|; phi = |x| - R.  With exact interpolation the
    foot points of eq. (SL2d)/(SL3d) sit at radius sqrt((r + c dt)^2 + m a^2),
    m = 1 (2D) or 2 (3D), a^2 = c delta r dt / p; at nodes with |phi| <= beta
    (c = 1) the scheme must converge to that value at the interpolant's order."""
    R = 0.5
    errs = []
    for n in (33, 65) if dim == 3 else (65, 129):
        g = _grid(dim, n)
        h = g["h"]
        prm = _params(dim, h)
        dt = 0.5 * h
        d = oracle.distance_brute(np.zeros((1, dim)), g)
        r = d.ravel()
        phi = (d - R)
        sel = np.nonzero((np.abs(phi.ravel()) <= prm["beta"]) & (r > 0.2))[0]
        got, flags = oracle.sl_nodes(phi, d, g, prm, dt, kind, sel)
        assert not (flags & 1).any()  # no fallback; the regularised frame is still tangent
        m = 1 if dim == 2 else 2
        a2 = prm["delta"] * r[sel] * dt / prm["p"]
        want = np.sqrt((r[sel] + dt) ** 2 + m * a2) - R
        errs.append(np.abs(got - want).max())
    assert errs[0] / errs[1] > min_ratio, errs
    assert errs[1] < 0.02 * h


def test_diffusion_amplitude_is_as_printed():
    """A wrong diffusion scale would leave an O(h) residual in the radial test:
    at a single node, compare with the closed form for several scales."""
    g = _grid(3, 65)
    h = g["h"]
    prm = _params(3, h)
    dt = 0.5 * h
    d = oracle.distance_brute(np.zeros((1, 3)), g)
    phi = d - 0.5
    sel = np.nonzero((np.abs(phi.ravel()) <= prm["beta"]) & (d.ravel() > 0.2))[0][:200]
    got, _ = oracle.sl_nodes(phi, d, g, prm, dt, "weno", sel)
    r = d.ravel()[sel]
    errs = {}
    for scale in (0.5, 1.0, 2.0):
        want = np.sqrt((r + dt) ** 2 + 2 * scale * r * dt) - 0.5
        errs[scale] = np.abs(got - want).max()
    assert errs[1.0] < 0.1 * min(errs[0.5], errs[2.0])


def test_regularised_frame_when_d1_and_d3_vanish():
    """At a node where d1 phi = d3 phi = 0 the 3D frame is (e1, e3) (Section 3.1)."""
    n = 21
    g = _grid(3, n)
    h = g["h"]
    X = oracle.node_coords(g)
    kappa = 0.8
    phi = (X[:, 1] + 0.5 * kappa * (X[:, 0] ** 2 + X[:, 2] ** 2)).reshape(g["n"])
    Dconst = 0.3
    d = np.full(g["n"], Dconst)
    prm = _params(3, h, gamma=50.0, beta=40.0)
    dt = 0.5 * h
    c = (10, 12, 10)  # x = 0, z = 0
    idx = np.ravel_multi_index(c, g["n"])
    got, flags = oracle.sl_nodes(phi, d, g, prm, dt, "weno", [idx])
    assert flags[0] & 2
    a2 = Dconst * dt
    y = X[idx, 1]
    # foot points (+-a, y, +-a): phi = y + kappa a^2 exactly (quadratic, WENO exact)
    assert got[0] == pytest.approx(y + kappa * a2, abs=1e-12)


def test_fallback_on_flat_gradient():
    g = _grid(2, 9)
    h = g["h"]
    X = oracle.node_coords(g)
    phi = (0.01 * (X[:, 0] ** 2 + X[:, 1] ** 2)).reshape(g["n"])
    d = np.full(g["n"], 0.4)
    prm = _params(2, h, gamma=1.0, beta=0.5)
    idx = np.ravel_multi_index((4, 4), g["n"])  # the origin: centred gradient 0
    got, flags = oracle.sl_nodes(phi, d, g, prm, h, "q1", [idx])
    assert flags[0] & 1
    assert got[0] == pytest.approx(0.01 * h * h, abs=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_phi_stays_constant(dim):
    g = _grid(dim, 8)
    phi = np.full(g["n"], 0.01)
    d = np.full(g["n"], 0.3)
    prm = _params(dim, g["h"])
    out, band, counts = oracle.step(phi, d, g, prm, g["h"], "weno")
    assert band.all() and counts[1] == band.size
    np.testing.assert_array_equal(out, phi)


def test_mirror_symmetry_of_a_step():
    """Inputs symmetric under x -> -x give an output symmetric under it."""
    g = _grid(3, 25)
    h = g["h"]
    prm = _params(3, h)
    phi = oracle.init_phi(g, "sphere", (0, 0, 0, 0.7), prm["gamma"])
    X = oracle.node_coords(g)
    d = np.abs(np.linalg.norm(X, axis=1) - 0.4).reshape(g["n"])
    for kind in ("q1", "weno"):
        out, _, _ = oracle.step(phi, d, g, prm, 0.5 * h, kind)
        np.testing.assert_allclose(out, out[::-1, :, :], atol=1e-13)
        np.testing.assert_allclose(out, out[:, :, ::-1], atol=1e-13)


def test_band_and_cut():
    g = _grid(3, 20)
    h = g["h"]
    prm = _params(3, h)
    phi = oracle.init_phi(g, "sphere", (0.05, 0, 0, 0.6), prm["gamma"])
    pts = np.random.default_rng(3).normal(size=(100, 3))
    pts = 0.3 * pts / np.linalg.norm(pts, axis=1, keepdims=True)
    d = oracle.distance_brute(pts, g)
    out, band, counts = oracle.step(phi, d, g, prm, 0.5 * h, "weno")
    np.testing.assert_array_equal(band, np.abs(phi) < prm["gamma"])
    assert counts[0] == band.sum()
    np.testing.assert_array_equal(out[band == 0], phi[band == 0])
    assert np.abs(out).max() <= prm["gamma"]


def test_restart_preserves_the_run():
    g = _grid(2, 40)
    h = g["h"]
    prm = _params(2, h, reinit_every=3)
    phi0 = oracle.init_phi(g, "sphere", (0, 0, 0, 0.8), prm["gamma"])
    pts = np.stack([0.4 * np.cos(np.linspace(0, 6, 30)), 0.4 * np.sin(np.linspace(0, 6, 30))], 1)
    d = oracle.distance_brute(pts, g)
    full, c_full = oracle.run(phi0, d, g, prm, h, "weno", 10)
    half, c1 = oracle.run(phi0, d, g, prm, h, "weno", 4)
    rest, c2 = oracle.run(half, d, g, prm, h, "weno", 6, step0=4)
    np.testing.assert_array_equal(full, rest)
    assert c_full[0] == c1[0] + c2[0] and c_full[3] == c1[3] + c2[3] == 3


# ------------------------------------------------------------- distance

@pytest.mark.parametrize("dim", [2, 3])
def test_distance_kdtree_matches_brute_force(dim):
    g = _grid(dim, 17 if dim == 3 else 40)
    pts = RNG.uniform(-0.8, 0.8, size=(150, dim))
    np.testing.assert_allclose(oracle.distance(pts, g), oracle.distance_brute(pts, g),
                               rtol=0, atol=1e-15)


def test_distance_single_point_is_euclidean():
    g = _grid(3, 9)
    q = np.array([[0.123, -0.456, 0.789]])
    d = oracle.distance_brute(q, g).ravel()
    X = oracle.node_coords(g)
    for j in range(0, len(X), 37):
        want = math.sqrt(sum((X[j, a] - q[0, a]) ** 2 for a in range(3)))
        assert d[j] == pytest.approx(want, rel=1e-15)


# --------------------------------------------------------- initial data

def _surface_distance(X, surf):
    from scipy.spatial import cKDTree
    return cKDTree(surf).query(X)[0]


def test_initial_sphere_and_torus_are_signed_distances():
    g = _grid(3, 21)
    X = oracle.node_coords(g)
    rng = np.random.default_rng(7)
    # dense surface samples; |phi| must be their distance up to sampling error
    u = rng.normal(size=(400_000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    c, R = np.array([0.1, -0.05, 0.02]), 0.55
    phi = oracle.init_phi(g, "sphere", (*c, R), 10.0).ravel()
    ds = _surface_distance(X, c + R * u)
    assert np.abs(np.abs(phi) - ds).max() < 5e-3
    inside = np.linalg.norm(X - c, axis=1) < R
    assert (phi[inside] < 0).all() and (phi[~inside] > 0).all()
    a, b = rng.uniform(0, 2 * np.pi, (2, 600_000))
    Rt, rt = 0.5, 0.2
    surf = np.stack([(Rt + rt * np.cos(b)) * np.cos(a), (Rt + rt * np.cos(b)) * np.sin(a),
                     rt * np.sin(b)], 1)
    phi = oracle.init_phi(g, "torus", (0, 0, 0, Rt, rt), 10.0).ravel()
    ds = _surface_distance(X, surf)
    assert np.abs(np.abs(phi) - ds).max() < 5e-3
    gam = 0.2
    phic = oracle.init_phi(g, "torus", (0, 0, 0, Rt, rt), gam)
    assert np.abs(phic).max() <= gam
