"""Pins of the oracle's multi-run schedule (Section 4: Table param, eq. dxdt,
the warm start of each finer run from the previous steady state).

The grid of each run is a reading (the paper only says that the grid
encompasses the cloud); it is pinned by the grid sizes the paper prints for
its 64-point circle.  The warm start is the run's interpolator applied to
the previous result, pinned by the exactness of Q1 on multilinear and of
WENO on tensor-quadratic data.  The whole schedule on the paper's circle is
held to the paper's printed errors within a factor of two (the readings of
the reinitialisation and of the band make the exact values differ).
"""
import math

import numpy as np
import pytest

import oracle
from conftest import read_golden_values

GOLD = read_golden_values("schedule.txt")


def circle64():
    th = np.arange(64) * (2.0 * np.pi / 64)
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def test_table_param():
    for r in (1, 2, 3):
        assert oracle.run_params(r) == (GOLD[f"run{r}_p"], GOLD[f"run{r}_delta"])
    for r in (4, 7):
        assert oracle.run_params(r) == oracle.run_params(3)
    with pytest.raises(ValueError):
        oracle.run_params(0)


def test_spacing_halves_per_run_and_dt_is_a_quarter():
    hs = 0.137
    for r in range(1, 6):
        dx, dt = oracle.run_spacing(hs, r)
        assert dx == hs / 2 ** (r - 1) and dt == dx / 4


def test_circle_grid_sizes_from_the_paper():
    pts = circle64()
    hs = oracle.cloud_spacing(pts, np.arange(64))
    assert hs == pytest.approx(2 * math.sin(math.pi / 64), rel=1e-12)
    for r in range(1, 6):
        g = oracle.run_grid(pts, hs, r)
        n = int(GOLD[f"circle64_grid_r{r}"])
        assert g["n"] == (n, n), (r, g["n"])
        # the grid holds the cloud with the margin on every side
        m = oracle.run_margin(2, hs, r)
        top = np.asarray(g["lo"]) + (np.asarray(g["n"]) - 1) * g["h"]
        assert (np.asarray(g["lo"]) <= pts.min(0) - m * g["h"] + 1e-12).all()
        assert (top >= pts.max(0) + m * g["h"] - 1e-12).all()


def test_first_margin_adds_gamma_s():
    # K_S = 2 adds two cells of h_S to the first run only; a larger K_S more
    assert oracle.run_margin(3, 0.1, 1) == 12 and oracle.run_margin(3, 0.1, 2) == 10
    assert oracle.run_margin(3, 0.1, 1, K_S=5.0) == 15
    assert oracle.run_margin(2, 0.1, 1) == 10 and oracle.run_margin(2, 0.1, 3) == 8


def _grid(dim, n, h, lo):
    return {"dim": dim, "n": (n,) * dim, "lo": (lo,) * dim, "h": h}


@pytest.mark.parametrize("dim", [2, 3])
def test_resample_exact_on_the_interpolators_polynomials(dim):
    coarse = _grid(dim, 13, 0.2, -1.2)
    fine = _grid(dim, 19, 0.1, -0.9)
    Xc, Xf = oracle.node_coords(coarse), oracle.node_coords(fine)
    rng = np.random.default_rng(5)
    # multilinear data: Q1 reproduces it exactly
    a = rng.normal(size=dim)
    lin = lambda X: 0.3 + X @ a + 0.7 * np.prod(X, axis=1)
    got = oracle.resample(lin(Xc).reshape(coarse["n"]), coarse, fine, "q1")
    np.testing.assert_allclose(got.ravel(), lin(Xf), atol=1e-12)
    # tensor-quadratic data: WENO reproduces it exactly (stencils inside)
    quad = lambda X: 0.2 + np.sum(X * X, axis=1) + 0.5 * X[:, 0] * X[:, -1]
    got = oracle.resample(quad(Xc).reshape(coarse["n"]), coarse, fine, "weno")
    np.testing.assert_allclose(got.ravel(), quad(Xf), atol=1e-11)
    # but not Q1 on the quadratic: the interpolator matters
    got = oracle.resample(quad(Xc).reshape(coarse["n"]), coarse, fine, "q1")
    assert np.abs(got.ravel() - quad(Xf)).max() > 1e-3


def test_resample_keeps_coincident_nodes():
    coarse = _grid(2, 11, 0.2, -1.0)
    fine = _grid(2, 21, 0.1, -1.0)
    f = np.random.default_rng(3).normal(size=coarse["n"])
    for kind in ("q1", "weno"):
        got = oracle.resample(f, coarse, fine, kind)
        np.testing.assert_allclose(got[::2, ::2], f, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["q1", "weno"])
def test_three_runs_on_the_paper_circle(kind):
    """The paper's 2D circle test, three runs: the grids of the table, a
    steady state in every run within the stopping test's 10..100 steps, and
    the final L1 error (over the band of the exact distance) and cloud error
    within a factor two of the values the paper prints."""
    pts = circle64()
    hs, runs = oracle.reconstruct(pts, np.arange(64), kind, runs=3)
    for r, run in enumerate(runs, 1):
        n = int(GOLD[f"circle64_grid_r{r}"])
        assert run["grid"]["n"] == (n, n)
        assert 10 <= run["steps"] < 100
        assert (run["params"]["p"], run["params"]["delta"]) == oracle.run_params(r)
    last = runs[-1]
    g = last["grid"]
    exact = (np.linalg.norm(oracle.node_coords(g), axis=1) - 1.0).reshape(g["n"])
    near = np.abs(exact) < last["params"]["gamma"]
    l1 = float(np.abs(last["phi"] - exact)[near].sum() * g["h"] ** 2)
    err_s = float(np.mean(np.abs(oracle.interp(last["phi"], g, pts, "q1"))))
    want_l1, want_s = GOLD[f"circle64_r3_L1_{kind}"], GOLD[f"circle64_r3_errS_{kind}"]
    assert want_l1 / 2 < l1 < 2 * want_l1, l1
    assert want_s / 2 < err_s < 2 * want_s, err_s
    # the warm start carries the previous run's front: the first energy of
    # a run is close to the last of the one before
    for a, b in zip(runs, runs[1:]):
        assert abs(b["energies"][0] - a["energies"][-1]) < 0.25 * a["energies"][-1]
