"""Pins of the oracle's interpolators (Section 3.2) against facts the paper and
the mathematics fix: printed linear weights and indicator matrices, the
indicator's integral definition, polynomial exactness, order of accuracy,
symmetry and continuity."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

import oracle
from conftest import read_golden_matrices, read_golden_values

RNG = np.random.default_rng(1234)


def test_weno_linear_weights_match_paper():
    gold = read_golden_values("weno_linear_weights.txt")
    for s, key in [(-1.0, "s=-1"), (0.0, "s=0"), (2.0, "s=2")]:
        _, parts = oracle.weno1d([0.0, 0.0, 0.0, 0.0], s, 1.0, parts=True)
        if f"C_L({key})" in gold:
            assert parts["CL"] == pytest.approx(gold[f"C_L({key})"], abs=1e-15)
        if f"C_R({key})" in gold:
            assert parts["CR"] == pytest.approx(gold[f"C_R({key})"], abs=1e-15)
    # C_k(x) = gamma_k (x - xhat_k)/dx with xhat_L = x_{j+2}, xhat_R = x_{j-1}
    for s in np.linspace(0.0, 1.0, 7):
        _, parts = oracle.weno1d([0.0] * 4, s, 1.0, parts=True)
        assert parts["CL"] == pytest.approx(gold["gamma_L"] * (s - 2.0), abs=1e-15)
        assert parts["CR"] == pytest.approx(gold["gamma_R"] * (s + 1.0), abs=1e-15)
        assert parts["CL"] + parts["CR"] == pytest.approx(1.0, abs=1e-15)


def test_weno_indicators_match_printed_matrices():
    mats = read_golden_matrices("weno_indicator_matrices.txt")
    AL, AR = np.array(mats["A_L"]), np.array(mats["A_R"])
    for _ in range(50):
        v = RNG.normal(size=4)
        dx = RNG.uniform(0.01, 2.0)
        _, parts = oracle.weno1d(v, RNG.uniform(), dx, parts=True)
        assert parts["IL"] == pytest.approx(v @ AL @ v / dx ** 2, rel=1e-12)
        assert parts["IR"] == pytest.approx(v @ AR @ v / dx ** 2, rel=1e-12)


def test_weno_indicators_match_integral_definition():
    """eq. (ind:1d): I[P] = sum_{b>=2} dx^(2b-3) int_{x_j}^{x_{j+1}} (P^(b))^2 dx,
    evaluated with NumPy's polynomial fit and exact integration."""
    for _ in range(20):
        dx = RNG.uniform(0.05, 1.5)
        xj = RNG.uniform(-1, 1)
        xs = xj + dx * np.array([-1.0, 0.0, 1.0, 2.0])
        v = RNG.normal(size=4)
        _, parts = oracle.weno1d(v, 0.3, dx, parts=True)
        for key, sel in [("IL", slice(0, 3)), ("IR", slice(1, 4))]:
            c = Pn.polyfit(xs[sel], v[sel], 2)
            total = 0.0
            for b in (2, 3):
                der = Pn.polyder(c, b)
                sq = Pn.polyint(Pn.polymul(der, der))
                total += dx ** (2 * b - 3) * (Pn.polyval(xj + dx, sq) - Pn.polyval(xj, sq))
            assert parts[key] == pytest.approx(total, rel=1e-9, abs=1e-12)


def test_weno_polynomials_interpolate_their_substencils():
    for _ in range(20):
        v = RNG.normal(size=4)
        for s, iL, iR in [(-1.0, 0, None), (0.0, 1, 0), (1.0, 2, 1), (2.0, None, 2)]:
            _, parts = oracle.weno1d(v, s, 0.7, parts=True)
            if iL is not None:
                assert parts["PL"] == pytest.approx(v[iL], abs=1e-13)
            if iR is not None:
                assert parts["PR"] == pytest.approx(v[iR + 1], abs=1e-13)


def test_weno_exact_on_quadratics_not_on_cubics():
    for _ in range(50):
        dx = RNG.uniform(0.01, 1.0)
        c = RNG.normal(size=3)
        xs = dx * np.array([-1.0, 0.0, 1.0, 2.0])
        s = RNG.uniform()
        got = oracle.weno1d(Pn.polyval(xs, c), s, dx)
        assert got == pytest.approx(Pn.polyval(s * dx, c), abs=1e-12)
    # a cubic with a sizeable third derivative is not reproduced
    dx = 0.5
    xs = dx * np.array([-1.0, 0.0, 1.0, 2.0])
    c = [0.1, -0.3, 0.2, 4.0]
    got = oracle.weno1d(Pn.polyval(xs, c), 0.4, dx)
    assert abs(got - Pn.polyval(0.4 * dx, c)) > 1e-4


def test_weno_smooth_limit_is_cubic_lagrange():
    """When the indicators are negligible against eps the weights are the
    linear ones and sum_k C_k P_k is the cubic through the four nodes."""
    dx = 1.0
    xs = dx * np.array([-1.0, 0.0, 1.0, 2.0])
    c = 1e-7 * np.array([0.3, -1.0, 0.5, 2.0])
    v = Pn.polyval(xs, c)
    for s in np.linspace(0, 1, 9):
        got = oracle.weno1d(v, s, dx)
        assert got == pytest.approx(Pn.polyval(s * dx, c), rel=1e-9, abs=1e-20)


def test_weno_mirror_symmetry():
    for _ in range(50):
        v = RNG.normal(size=4)
        s = RNG.uniform()
        assert oracle.weno1d(v, s, 0.3) == pytest.approx(oracle.weno1d(v[::-1], 1.0 - s, 0.3),
                                                         abs=1e-13)


def test_weno_observed_order_on_smooth_data():
    errs = []
    for n in (16, 32, 64, 128):
        dx = 1.0 / n
        worst = 0.0
        for x in np.linspace(0.1, 0.9, 37):
            j = int(np.floor(x / dx))
            s = x / dx - j
            xs = dx * (j + np.array([-1, 0, 1, 2]))
            worst = max(worst, abs(oracle.weno1d(np.sin(3 * xs), s, dx) - np.sin(3 * x)))
        errs.append(worst)
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert min(ratios) > 2 ** 3 * 0.9, (errs, ratios)


def _grid(dim, n, lo=-1.0, hi=1.0):
    return {"dim": dim, "n": (n,) * dim, "lo": (lo,) * dim, "h": (hi - lo) / (n - 1)}


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_exact_on_multilinear(dim):
    g = _grid(dim, 9)
    X = oracle.node_coords(g)
    coef = RNG.normal(size=2 ** dim)

    def f(P):
        out = np.zeros(len(P))
        for m in range(2 ** dim):
            term = coef[m] * np.ones(len(P))
            for a in range(dim):
                if (m >> a) & 1:
                    term *= P[:, a]
            out += term
        return out

    vals = f(X).reshape(g["n"])
    pts = RNG.uniform(-1, 1, size=(40, dim))
    got = oracle.interp(vals, g, pts, "q1")
    np.testing.assert_allclose(got, f(pts), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["q1", "weno"])
def test_interpolants_reproduce_nodes(dim, kind):
    g = _grid(dim, 7)
    vals = RNG.normal(size=g["n"])
    X = oracle.node_coords(g)
    sel = RNG.choice(len(X), size=25, replace=False)
    got = oracle.interp(vals, g, X[sel], kind)
    np.testing.assert_allclose(got, vals.ravel()[sel], atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_is_a_convex_combination(dim):
    g = _grid(dim, 6)
    vals = RNG.normal(size=g["n"])
    pts = RNG.uniform(-1, 1, size=(60, dim))
    got = oracle.interp(vals, g, pts, "q1")
    assert got.max() <= vals.max() + 1e-14 and got.min() >= vals.min() - 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_tensor_weno_exact_on_tensor_quadratics(dim):
    g = _grid(dim, 10)
    X = oracle.node_coords(g)
    # random polynomial of degree <= 2 in every variable separately
    C = RNG.normal(size=(3,) * dim)

    def f(P):
        out = np.zeros(len(P))
        for e in np.ndindex(*C.shape):
            term = C[e] * np.ones(len(P))
            for a in range(dim):
                term *= P[:, a] ** e[a]
            out += term
        return out

    vals = f(X).reshape(g["n"])
    lo = -1 + 1.01 * g["h"]
    pts = RNG.uniform(lo, -lo, size=(40, dim))  # keep the 4-wide stencil inside
    got = oracle.interp(vals, g, pts, "weno")
    np.testing.assert_allclose(got, f(pts), atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_tensor_weno_continuous_across_faces(dim):
    g = _grid(dim, 8)
    vals = RNG.normal(size=g["n"])
    for _ in range(20):
        p = RNG.uniform(-0.7, 0.7, size=dim)
        a = int(RNG.integers(dim))
        face = -1 + g["h"] * np.round((p[a] + 1) / g["h"])
        lo_pt, hi_pt = p.copy(), p.copy()
        lo_pt[a] = face - 1e-11
        hi_pt[a] = face + 1e-11
        got = oracle.interp(vals, g, np.stack([lo_pt, hi_pt]), "weno")
        assert abs(got[0] - got[1]) < 1e-8


def test_tensor_weno_last_axis_first_2d():
    """Section 3.2: in 2D four WENO interpolations along y give auxiliary data
    in x, then one WENO along x.  Built here from the 1D routine."""
    g = _grid(2, 8)
    vals = RNG.normal(size=g["n"])
    h = g["h"]
    for _ in range(10):
        p = RNG.uniform(-0.6, 0.6, size=2)
        u = (p + 1) / h
        i0 = np.floor(u).astype(int)
        t = u - i0
        w = [oracle.weno1d(vals[i0[0] - 1 + a, i0[1] - 1:i0[1] + 3], t[1], h) for a in range(4)]
        want = oracle.weno1d(np.array(w), t[0], h)
        got = oracle.interp(vals, g, p[None], "weno")[0]
        assert got == pytest.approx(want, abs=1e-14)
        # x first gives another value: the one-dimensional WENO is nonlinear
        wx = [oracle.weno1d(vals[i0[0] - 1:i0[0] + 3, i0[1] - 1 + b], t[0], h) for b in range(4)]
        assert abs(oracle.weno1d(np.array(wx), t[1], h) - got) > 1e-6


def _weno3_in_order(vals, i0, t, h, order):
    """Tensor WENO at a point from the 1D routine, reducing the axes in the
    given order (the first axis of `order` is interpolated first)."""
    block = vals[i0[0] - 1:i0[0] + 3, i0[1] - 1:i0[1] + 3, i0[2] - 1:i0[2] + 3]
    axes = list(range(3))
    for ax in order:
        pos = axes.index(ax)
        block = np.apply_along_axis(lambda v: oracle.weno1d(v, t[ax], h), pos, block)
        axes.pop(pos)
    return float(block)


def test_tensor_weno_last_axis_first_3d():
    """Section 3.2 extended to 3D by analogy: WENO along z first (16 lines),
    then y (4 lines), then x.  Every other order gives a different value on
    rough data, so an oracle that reduced the axes in another order fails
    here although exactness on tensor quadratics and continuity hold for any
    order."""
    g = _grid(3, 8)
    vals = RNG.normal(size=g["n"])
    h = g["h"]
    others = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1)]
    for _ in range(10):
        p = RNG.uniform(-0.6, 0.6, size=3)
        u = (p + 1) / h
        i0 = np.floor(u).astype(int)
        t = u - i0
        got = oracle.interp(vals, g, p[None], "weno")[0]
        assert got == pytest.approx(_weno3_in_order(vals, i0, t, h, (2, 1, 0)), abs=1e-14)
        for order in others:
            assert abs(_weno3_in_order(vals, i0, t, h, order) - got) > 1e-6, order


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["q1", "weno"])
def test_constant_stencils_are_returned_exactly(dim, kind):
    """Both interpolants reproduce constants (eqs. (IQ1), (IWENO)); the
    oracle evaluates them so that this holds bit for bit, which fixes the
    value read from inside the cut plateau at exactly +-gamma."""
    g = _grid(dim, 9)
    for c in (6 * 2.0 / 127, -0.0470588235294118, 0.3):
        vals = np.full(g["n"], c)
        pts = RNG.uniform(-1, 1, size=(200, dim))
        got = oracle.interp(vals, g, pts, kind)
        assert (got == c).all()
    for s in RNG.uniform(0, 1, size=50):
        v = np.full(4, 0.0472440944881889)
        r, parts = oracle.weno1d(v, s, 0.1, parts=True)
        assert r == v[0] and parts["wL"] + parts["wR"] == 1.0
