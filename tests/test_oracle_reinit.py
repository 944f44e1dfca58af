"""Pins of the oracle's reinitialisation (Section 3.7 on the band of Section
3.8).  The paper defines it only by reference, so the oracle follows a stated
reading; these tests pin that reading against properties any consistent
reinitialisation must have (a planar signed distance is a fixed point; the
steady state is a signed distance; the zero set stays put) and against the
closed-form recursion the upwind forward-Euler update reduces to for a plane
normal to a grid axis."""
import math

import numpy as np
import pytest

import oracle


def _grid(dim, n, lo=-1.0, hi=1.0):
    return {"dim": dim, "n": (n,) * dim, "lo": (lo,) * dim, "h": (hi - lo) / (n - 1)}


@pytest.mark.parametrize("dim", [2, 3])
def test_planar_signed_distance_is_a_fixed_point(dim):
    """A node's value after m iterations depends on nodes at most m cells
    away, so nodes farther than reinit_iters from the domain boundary never
    see the boundary rule (a missing neighbour contributes no difference)."""
    rng = np.random.default_rng(5 + dim)
    g = _grid(dim, 40 if dim == 3 else 48)
    h = g["h"]
    prm = oracle.default_params(dim, h)
    m = prm["reinit_iters"] + 1
    inner = (slice(m, -m),) * dim
    X = oracle.node_coords(g)
    for _ in range(3):
        nrm = rng.normal(size=dim)
        nrm /= np.linalg.norm(nrm)
        phi = np.clip(X @ nrm - 0.1 * rng.uniform(), -prm["gamma"], prm["gamma"]).reshape(g["n"])
        band = oracle.band_mask(phi, prm)
        out, counts = oracle.reinit(phi, band, g, prm)
        assert counts[1] > 0 and band[inner].any()
        np.testing.assert_allclose(out[inner], phi[inner], atol=1e-13)


def _axis_plane_expected(phi_tilde_line, gamma, h, dtau, iters):
    """Reinitialisation along one axis for phi~ increasing in x: one-step fix
    exact on the two nodes that straddle the zero (centred gradient of a
    linear function), then, because the profile stays increasing, the upwind
    update reduces to phi_j <- phi_j - dtau*(phi_j - phi_{j-1} - h)/h on the
    positive side and phi_j <- phi_j + dtau*(phi_{j+1} - phi_j - h)/h on the
    negative side."""
    f = phi_tilde_line.copy()
    n = len(f)
    band = np.abs(f) < gamma
    gbar = band.copy()
    gbar[1:] |= band[:-1]
    gbar[:-1] |= band[1:]
    itf = np.zeros(n, bool)
    for j in range(n):
        for k in (j - 1, j + 1):
            if 0 <= k < n and gbar[j] and f[j] * f[k] <= 0:
                itf[j] = True
    cur = f.copy()
    for j in np.nonzero(itf)[0]:
        cur[j] = f[j] / ((f[j + 1] - f[j - 1]) / (2 * h))
    for _ in range(iters):
        nxt = cur.copy()
        for j in np.nonzero(gbar & ~itf)[0]:
            if f[j] > 0:
                assert cur[j] >= cur[j - 1]
                nxt[j] = cur[j] - dtau * ((cur[j] - cur[j - 1]) / h - 1.0)
            elif f[j] < 0:
                assert cur[j + 1] >= cur[j]
                nxt[j] = cur[j] + dtau * ((cur[j + 1] - cur[j]) / h - 1.0)
        cur = nxt
    out = f.copy()
    out[gbar] = np.clip(cur[gbar], -gamma, gamma)
    return out


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("slope", [2.0, 0.5])
def test_axis_plane_follows_the_upwind_recursion(dim, slope):
    g = _grid(dim, 30)
    h = g["h"]
    prm = oracle.default_params(dim, h)
    X = oracle.node_coords(g)
    x0 = 0.0371
    phi = np.clip(slope * (X[:, 0] - x0), -prm["gamma"], prm["gamma"]).reshape(g["n"])
    band = oracle.band_mask(phi, prm)
    out, _ = oracle.reinit(phi, band, g, prm)
    line = phi[(slice(None),) + (5,) * (dim - 1)]
    want = _axis_plane_expected(line, prm["gamma"], h, prm["reinit_dtau"], prm["reinit_iters"])
    for sl in [(slice(None),) + (5,) * (dim - 1), (slice(None),) + (11,) * (dim - 1)]:
        np.testing.assert_allclose(out[sl], want, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_steady_state_is_the_signed_distance(dim):
    """Run to (near) steady state: a plane with |grad| = 2 becomes its signed
    distance on the reinitialisation band.  At steady state a node depends only
    on nodes along its backward characteristic, at most |SDF|/h <= 5 cells long
    on this band, so a 6-cell margin keeps the domain-boundary rule out."""
    rng = np.random.default_rng(11)
    g = _grid(dim, 30)
    h = g["h"]
    X = oracle.node_coords(g)
    nrm = rng.normal(size=dim)
    nrm /= np.linalg.norm(nrm)
    sdf = (X @ nrm - 0.05).reshape(g["n"])
    prm = oracle.default_params(dim, h, reinit_iters=300)
    phi = np.clip(2.0 * sdf, -prm["gamma"], prm["gamma"])
    band = oracle.band_mask(phi, prm)
    out, _ = oracle.reinit(phi, band, g, prm)
    gb = band.astype(bool)
    for a in range(dim):
        gb = gb | np.roll(band, 1, axis=a).astype(bool) | np.roll(band, -1, axis=a).astype(bool)
    inner = np.zeros(g["n"], bool)
    inner[(slice(6, -6),) * dim] = True
    sel = gb & inner
    np.testing.assert_allclose(out[sel], sdf[sel], atol=1e-10)


def test_sphere_change_vanishes_with_h():
    """Exact sphere SDF: the first-order scheme moves it by O(h^2), i.e. the
    change in units of h vanishes linearly."""
    rel = []
    for n in (33, 65):
        g = _grid(3, n)
        h = g["h"]
        prm = oracle.default_params(3, h)
        phi = oracle.init_phi(g, "sphere", (0.01, -0.02, 0.03, 0.55), prm["gamma"])
        band = oracle.band_mask(phi, prm)
        out, _ = oracle.reinit(phi, band, g, prm)
        rel.append(np.abs(out - phi).max() / h)
    # first order: the change measured in cells halves with h
    assert rel[1] < 0.6 * rel[0], rel


def _edge_crossings(phi, axis):
    a = np.moveaxis(phi, axis, 0)
    s0, s1 = a[:-1], a[1:]
    cross = (s0 * s1 < 0)
    t = np.where(cross, s0 / np.where(cross, s0 - s1, 1.0), 0.0)
    return cross, t


def test_zero_set_stays_put():
    """phi~ = g * SDF with g smooth and positive: the sign pattern is kept and
    the linear edge crossings move by a small fraction of h."""
    n = 49
    g = _grid(3, n)
    h = g["h"]
    prm = oracle.default_params(3, h)
    X = oracle.node_coords(g)
    sdf = (np.linalg.norm(X - np.array([0.02, 0.01, -0.03]), axis=1) - 0.5)
    gfac = 1.0 + 0.4 * X[:, 0] + 0.2 * X[:, 1] ** 2
    phi = np.clip((gfac * sdf).reshape(g["n"]), -prm["gamma"], prm["gamma"])
    band = oracle.band_mask(phi, prm)
    out, _ = oracle.reinit(phi, band, g, prm)
    np.testing.assert_array_equal(np.sign(out), np.sign(phi))
    for ax in range(3):
        c0, t0 = _edge_crossings(phi, ax)
        c1, t1 = _edge_crossings(out, ax)
        np.testing.assert_array_equal(c0, c1)
        assert np.abs(t0 - t1)[c0].max() < 0.05
    # and the result is much closer to a distance than the input
    sd = sdf.reshape(g["n"])
    near = np.abs(sd) < 3 * h
    assert np.abs(out - sd)[near].max() < 0.25 * np.abs(phi - sd)[near].max()
    assert math.isfinite(float(out.sum()))
