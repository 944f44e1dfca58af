"""FP64 CPU oracle for the narrow-band semi-Lagrangian level-set method of
Preda & Semplice (arXiv:2410.22205).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library: the arithmetic lives in ``lsr_oracle.c`` (plain C,
double precision, one node at a time) and is reached through ctypes; the exact
distance field for large grids uses SciPy's k-d tree nearest-neighbour query
(a library primitive) and is pinned against brute force in the tests.

Every function takes plain NumPy arrays.  Grids are dicts
``{"dim": 2|3, "n": (n0, n1[, n2]), "lo": (..), "h": h}`` and parameters are
dicts with the keys of :data:`PARAM_KEYS` (see :func:`default_params`).
Nodal arrays are C-ordered with shape ``n`` (axis 0 <-> x).
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("h", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("delta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("grad_C", ctypes.c_double), ("grad_alpha", ctypes.c_double),
                ("energy", ctypes.c_double),
                ("reinit_every", ctypes.c_int32), ("reinit_iters", ctypes.c_int32),
                ("reinit_dtau", ctypes.c_double), ("interface_floor", ctypes.c_double)]


PARAM_KEYS = [f[0] for f in _Params._fields_]

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_GP = ctypes.POINTER(_Grid)
_PP = ctypes.POINTER(_Params)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        sig = {
            "orc_cutoff": (ctypes.c_double, [ctypes.c_double] * 3),
            "orc_energy_sum": (ctypes.c_double, [_D, _D, _GP, ctypes.c_double, ctypes.c_int]),
            "orc_phi0_from_cloud": (ctypes.c_int, [_D, _GP, ctypes.c_double, ctypes.c_int, _D,
                                                   _U8]),
            "orc_distance_approx": (ctypes.c_int, [_D, ctypes.c_int64, _D, _GP, ctypes.c_int, _D,
                                                   _U8]),
            "orc_weno1d": (ctypes.c_double, [_D, ctypes.c_double, ctypes.c_double, _D]),
            "orc_interp": (ctypes.c_double, [_D, _GP, ctypes.c_int, _D]),
            "orc_gradient": (None, [_D, _GP, ctypes.c_int64, _D]),
            "orc_sl_nodes": (None, [_D, _D, _GP, _PP, ctypes.c_double, ctypes.c_int, _I64,
                                    ctypes.c_int64, _D, _I32]),
            "orc_step": (None, [_D, _D, _GP, _PP, ctypes.c_double, ctypes.c_int, _D, _U8, _I64]),
            "orc_reinit": (None, [_D, _U8, _GP, _PP, _I64]),
            "orc_run": (None, [_D, _D, _GP, _PP, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                               ctypes.c_int32, _I64]),
            "orc_init_phi": (None, [_D, _GP, ctypes.c_int, _D, ctypes.c_double]),
            "orc_distance_brute": (None, [_D, ctypes.c_int64, _GP, _D]),
            "orc_resample": (None, [_D, _GP, ctypes.c_int, _GP, _D]),
            "orc_threads": (ctypes.c_int, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _ptr(a, t=_D):
    return a.ctypes.data_as(t)


def _grid(grid):
    g = _Grid()
    g.dim = int(grid["dim"])
    n = list(grid["n"]) + [1] * (3 - len(grid["n"]))
    lo = list(grid["lo"]) + [0.0] * (3 - len(grid["lo"]))
    for a in range(3):
        g.n[a] = int(n[a])
        g.lo[a] = float(lo[a])
    g.h = float(grid["h"])
    return g


def _params(prm):
    p = _Params()
    for k in PARAM_KEYS:
        setattr(p, k, prm[k])
    return p


def shape(grid):
    return tuple(int(v) for v in grid["n"][: grid["dim"]])


def default_params(dim, h, **over):
    """The paper's parameter values (Sections 3.1, 3.7, 3.8) plus the stated
    readings: p = delta = 1, gamma = 4h / 6h and beta = 2h / 3h in 2D / 3D,
    C = 1e-3, alpha = 1, pseudo-time step h/2 and ceil((gamma + h)/dtau)
    iterations, reinitialisation after every step in 2D and every 10th in 3D."""
    gamma = (4.0 if dim == 2 else 6.0) * h
    prm = dict(p=1.0, delta=1.0, gamma=gamma, beta=gamma / 2.0, grad_C=1e-3, grad_alpha=1.0,
               energy=1.0, reinit_every=1 if dim == 2 else 10, reinit_iters=0,
               reinit_dtau=0.5 * h, interface_floor=1e-3)
    prm.update(over)
    if "reinit_iters" not in over:
        prm["reinit_iters"] = int(math.ceil((prm["gamma"] + h) / prm["reinit_dtau"] - 1e-9))
    return prm


def cutoff(phi, beta, gamma):
    return _lib().orc_cutoff(float(phi), float(beta), float(gamma))


def weno1d(v, s, dx, parts=False):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(8)
    r = _lib().orc_weno1d(_ptr(v), float(s), float(dx), _ptr(out))
    if parts:
        keys = ["PL", "PR", "CL", "CR", "IL", "IR", "wL", "wR"]
        return r, dict(zip(keys, out.tolist()))
    return r


def interp(f, grid, x, kind):
    """Interpolate nodal field f at the points x (m x dim); kind 'q1'|'weno'."""
    lib = _lib()
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = _grid(grid)
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    k = 0 if kind == "q1" else 1
    out = np.empty(len(x))
    for m in range(len(x)):
        pt = np.zeros(3)
        pt[: grid["dim"]] = x[m]
        out[m] = lib.orc_interp(_ptr(f), ctypes.byref(g), k, _ptr(pt))
    return out


def gradient(f, grid, idx):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(3)
    _lib().orc_gradient(_ptr(f), ctypes.byref(_grid(grid)), int(idx), _ptr(out))
    return out[: grid["dim"]]


def sl_nodes(phi, d, grid, prm, dt, kind, idx):
    """Updated values (with the cut) at the flat node indices idx, no band test.
    Returns (values, flags) with flag bit 1 = fallback, 2 = frame regularised."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    flags = np.empty(len(idx), dtype=np.int32)
    _lib().orc_sl_nodes(_ptr(phi), _ptr(d), ctypes.byref(_grid(grid)), ctypes.byref(_params(prm)),
                        float(dt), 0 if kind == "q1" else 1, _ptr(idx, _I64), len(idx), _ptr(out),
                        _ptr(flags, _I32))
    return out, flags


def step(phi, d, grid, prm, dt, kind):
    """One time step on the whole grid.  Returns (phi_new, band_mask, counts)
    with counts = [band size, fallbacks, frame regularisations]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty_like(phi)
    band = np.empty(phi.shape, dtype=np.uint8)
    counts = np.zeros(3, dtype=np.int64)
    _lib().orc_step(_ptr(phi), _ptr(d), ctypes.byref(_grid(grid)), ctypes.byref(_params(prm)),
                    float(dt), 0 if kind == "q1" else 1, _ptr(out), _ptr(band, _U8),
                    _ptr(counts, _I64))
    return out, band, counts


def reinit(phi, band, grid, prm):
    """Reinitialisation on the band plus its neighbours.  Returns
    (phi_new, [|Gbar|, |I|])."""
    phi = np.array(phi, dtype=np.float64, order="C", copy=True)
    band = np.ascontiguousarray(band, dtype=np.uint8)
    counts = np.zeros(2, dtype=np.int64)
    _lib().orc_reinit(_ptr(phi), _ptr(band, _U8), ctypes.byref(_grid(grid)),
                      ctypes.byref(_params(prm)), _ptr(counts, _I64))
    return phi, counts


def run(phi0, d, grid, prm, dt, kind, n_steps, step0=0):
    """n_steps of Algorithm 1's loop (energy omitted, p = 1).  Returns
    (phi, counts) with counts = [node updates, fallbacks, frame
    regularisations, reinitialisations, sum |Gbar|, sum |I|]."""
    phi = np.array(phi0, dtype=np.float64, order="C", copy=True)
    d = np.ascontiguousarray(d, dtype=np.float64)
    counts = np.zeros(6, dtype=np.int64)
    _lib().orc_run(_ptr(phi), _ptr(d), ctypes.byref(_grid(grid)), ctypes.byref(_params(prm)),
                   float(dt), 0 if kind == "q1" else 1, int(step0), int(n_steps),
                   _ptr(counts, _I64))
    return phi, counts


def run_p(phi0, d, grid, prm, dt, kind, n_steps, step0=0, R=5):
    """n_steps of Algorithm 1's loop with the energy step, for p != 1: at
    every step E_p of the current phi (Section 3.5, R subcells per axis in
    3D) enters the update's C, then the band, update and every
    reinit_every-th step the reinitialisation and cut, as in :func:`run`.
    Returns (phi, energies) with energies[s] = E_p(phi^s)."""
    phi = np.array(phi0, dtype=np.float64, order="C", copy=True)
    energies = []
    for s in range(n_steps):
        E = energy(phi, d, grid, prm["p"], R)
        energies.append(E)
        nxt, band, _ = step(phi, d, grid, dict(prm, energy=E), dt, kind)
        if prm["reinit_every"] > 0 and (step0 + s + 1) % prm["reinit_every"] == 0:
            nxt, _ = reinit(nxt, band, grid, prm)
        phi = nxt
    return phi, energies


def band_mask(phi, prm):
    """Narrow band of eq. (subgrid), read as |phi| < gamma."""
    return (np.abs(phi) < prm["gamma"]).astype(np.uint8)


def init_phi(grid, kind, args, gamma):
    """Closed-form SDF (kind 'sphere' or 'torus') cut to [-gamma, gamma]."""
    phi = np.empty(shape(grid), dtype=np.float64)
    a = np.zeros(8)
    a[: len(args)] = args
    _lib().orc_init_phi(_ptr(phi), ctypes.byref(_grid(grid)), 1 if kind == "sphere" else 2,
                        _ptr(a), float(gamma))
    return phi


def node_coords(grid):
    axes = [grid["lo"][a] + grid["h"] * np.arange(grid["n"][a]) for a in range(grid["dim"])]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def distance_brute(points, grid):
    """d(x) = min_Q |x - Q| at every node by brute force (Section 2)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    d = np.empty(shape(grid), dtype=np.float64)
    _lib().orc_distance_brute(_ptr(pts), len(pts), ctypes.byref(_grid(grid)), _ptr(d))
    return d


def distance(points, grid, x=None):
    """Exact distance to the cloud at every node (or at the points x), through
    SciPy's exact k-d tree nearest-neighbour query."""
    from scipy.spatial import cKDTree
    tree = cKDTree(np.asarray(points, dtype=np.float64))
    if x is None:
        dd, _ = tree.query(node_coords(grid), k=1, workers=-1)
        return dd.reshape(shape(grid))
    dd, _ = tree.query(np.asarray(x, dtype=np.float64), k=1, workers=-1)
    return dd


def energy(phi, d, grid, p, R=5):
    """E_p(phi) of Section 3.5 (eq. energyApprox in 2D, eq. energyApproxFiner
    with R subcells per axis in 3D), from nodal phi and d."""
    f = np.ascontiguousarray(phi, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    assert f.shape == shape(grid) and dd.shape == shape(grid)
    s = _lib().orc_energy_sum(_ptr(f), _ptr(dd), ctypes.byref(_grid(grid)), float(p), int(R))
    return s ** (1.0 / p)


def stop_rule(energies, n, min_steps=10, max_steps=100, tol=1e-4, window=10):
    """The stopping test of eq. (deltaEn) after iteration n, from
    energies[i] = E_2(phi^i), i = 0..n: with k = min(n, window) and
    e_m = mean(E_2(phi^(m-k+1)), ..., E_2(phi^m)), stop when
    |e_(n-1) - e_n| / e_n < tol, never before min_steps iterations and
    always at max_steps (reading: both averages use the same k, so the one
    at n - 1 reaches back to phi^0 while n <= window; a zero average
    stops)."""
    if n >= max_steps:
        return True
    if n < min_steps or n < 1:
        return False
    k = min(n, window)
    cur = sum(energies[n - k + 1: n + 1]) / k
    prev = sum(energies[n - k: n]) / k
    if not cur > 0.0:
        return True
    return abs(prev - cur) / cur < tol


def cloud_spacing(points, sample):
    """h_S of Section 4 (the text after eq. dxdt): the mean over the sampled
    points (indices into points) of the distance to their nearest neighbour
    in the cloud, i.e. the second smallest distance to the cloud counting the
    point itself (an exact duplicate is a neighbour at distance 0).  Uses
    SciPy's exact k-d tree query for the two nearest points."""
    from scipy.spatial import cKDTree
    pts = np.asarray(points, dtype=np.float64)
    tree = cKDTree(pts)
    dd, _ = tree.query(pts[np.asarray(sample, dtype=np.int64)], k=2)
    return float(np.mean(dd[:, 1]))


def phi0_from_cloud(d, grid, gamma_s, max_cycles=100):
    """phi0 of Section 3.6 from the distance field d and the threshold
    gamma_S: external marking from the grid's boundary, d - gamma_S there,
    fast sweeping inside, sign reversed inside.  Returns (phi0, external,
    sweep cycles used)."""
    dd = np.ascontiguousarray(d, dtype=np.float64)
    assert dd.shape == shape(grid)
    phi = np.empty_like(dd)
    ext = np.empty(dd.shape, dtype=np.uint8)
    cycles = _lib().orc_phi0_from_cloud(_ptr(dd), ctypes.byref(_grid(grid)), float(gamma_s),
                                        int(max_cycles), _ptr(phi), _ptr(ext, _U8))
    return phi, ext, cycles


def distance_approx(points, grid, max_cycles=100):
    """The paper's approximate distance field (Section 3.4): exact at the
    nodes of a 4^dim box around each cloud point, fast sweeping elsewhere.
    Returns (d, fixed mask, sweep cycles used)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    exact = distance(pts, grid)
    d = np.empty_like(exact)
    fixed = np.empty(exact.shape, dtype=np.uint8)
    cycles = _lib().orc_distance_approx(_ptr(pts), len(pts), _ptr(exact), ctypes.byref(_grid(grid)),
                                        int(max_cycles), _ptr(d), _ptr(fixed, _U8))
    return d, fixed, cycles


def threads(n=0):
    """Worker threads of the oracle's per-node loops (n < 1: leave as is);
    returns the count in effect."""
    return int(_lib().orc_threads(int(n)))


# ------------------------------------------------ the multi-run schedule

def run_params(r):
    """(p, delta) of run r >= 1 of Algorithm 1 (Section 4, Table param):
    (1, 0), then (2, 0), then (2, 1) for every later run."""
    if r < 1:
        raise ValueError("runs are numbered from 1")
    return (1.0, 0.0) if r == 1 else ((2.0, 0.0) if r == 2 else (2.0, 1.0))


def run_spacing(h_s, r):
    """(dx, dt) of run r, eq. (dxdt): dx = h_S / 2^(r-1), dt = dx / 4."""
    dx = h_s / 2.0 ** (r - 1)
    return dx, dx / 4.0


def run_margin(dim, h_s, r, K_S=2.0):
    """Nodes added on each side of the cloud's bounding box on the grid of
    run r.  The paper says only that the grid encompasses the cloud
    (Algorithm 1, step 1).  Reading, fitted to every grid size the paper
    prints (the circle and square tables and the 3D grid table, with K_S = 2
    and, for the scans with larger K_S, 5 or 10): the band half width in
    cells (4 in 2D, 6 in 3D) plus 4, and in the first run also the
    threshold gamma_S = K_S h_S in cells, rounded up."""
    dx, _ = run_spacing(h_s, r)
    m = (4 if dim == 2 else 6) + 4
    if r == 1:
        m += int(math.ceil(K_S * h_s / dx - 1e-9))
    return m


def run_grid(points, h_s, r, K_S=2.0):
    """Grid of run r: spacing dx of eq. (dxdt); per axis the cloud's
    extent L in whole cells, ceil(L / dx), plus one node and the margin
    of run_margin on each side; node 0 sits the margin below the cloud's
    smallest coordinate."""
    pts = np.asarray(points, dtype=np.float64)
    dim = pts.shape[1]
    dx, _ = run_spacing(h_s, r)
    m = run_margin(dim, h_s, r, K_S)
    lo = pts.min(axis=0)
    ext = pts.max(axis=0) - lo
    n = tuple(int(math.ceil(ext[a] / dx)) + 1 + 2 * m for a in range(dim))
    return {"dim": dim, "n": n, "lo": tuple(float(lo[a] - m * dx) for a in range(dim)), "h": dx}


def resample(f, grid_from, grid, kind):
    """Warm start of a finer run (Section 4, after eq. dxdt): the nodal field
    f of grid_from interpolated at every node of grid with the interpolator
    kind ('q1' or 'weno', Section 3.2)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == shape(grid_from)
    out = np.empty(shape(grid), dtype=np.float64)
    _lib().orc_resample(_ptr(f), ctypes.byref(_grid(grid_from)), 0 if kind == "q1" else 1,
                        ctypes.byref(_grid(grid)), _ptr(out))
    return out


def run_to_steady(phi0, d, grid, prm, dt, kind, R=5, min_steps=10, max_steps=100, tol=1e-4):
    """One run of Algorithm 1 until the stopping test of eq. (deltaEn):
    E_2 of phi^0 and of every new phi (R subcells per axis in 3D); each
    step takes E_p(phi^n) (= E_2 when p = 2; unused at p = 1), the band,
    the update and every reinit_every-th step the reinitialisation and cut.
    Returns (phi, energies, steps)."""
    phi = np.array(phi0, dtype=np.float64, order="C", copy=True)
    energies = [energy(phi, d, grid, 2.0, R)]
    n = 0
    while True:
        E = energies[-1] if prm["p"] == 2.0 else energy(phi, d, grid, prm["p"], R)
        nxt, band, _ = step(phi, d, grid, dict(prm, energy=E), dt, kind)
        if prm["reinit_every"] > 0 and (n + 1) % prm["reinit_every"] == 0:
            nxt, _ = reinit(nxt, band, grid, prm)
        phi = nxt
        n += 1
        energies.append(energy(phi, d, grid, 2.0, R))
        if stop_rule(energies, n, min_steps, max_steps, tol):
            return phi, energies, n


def reconstruct(points, sample, kind, runs=3, K_S=2.0, R=5, min_steps=10, max_steps=100,
                tol=1e-4):
    """Algorithm 1 run `runs` times from coarse to fine (Section 4): h_S from
    the sampled points; run r on the grid of run_grid with (p, delta) of
    Table param and (dx, dt) of eq. (dxdt); the exact distance field on each
    grid; phi^0 of the first run from the cloud with gamma_S = K_S h_S
    (Section 3.6), of every later run the previous result resampled; each
    phi^0 cut to [-gamma, gamma]; each run stepped to steady state.  Returns
    (h_S, a list of per-run dicts: grid, params, dt, phi, energies,
    steps)."""
    pts = np.asarray(points, dtype=np.float64)
    h_s = cloud_spacing(pts, sample)
    out = []
    for r in range(1, runs + 1):
        g = run_grid(pts, h_s, r, K_S)
        p, delta = run_params(r)
        dx, dt = run_spacing(h_s, r)
        prm = default_params(g["dim"], dx, p=p, delta=delta)
        d = distance(pts, g)
        if r == 1:
            phi0, _, _ = phi0_from_cloud(d, g, K_S * h_s)
        else:
            phi0 = resample(out[-1]["phi"], out[-1]["grid"], g, kind)
        phi0 = np.clip(phi0, -prm["gamma"], prm["gamma"])
        phi, energies, n = run_to_steady(phi0, d, g, prm, dt, kind, R, min_steps, max_steps, tol)
        out.append({"grid": g, "params": prm, "dt": dt, "phi0": phi0, "phi": phi,
                    "energies": energies, "steps": n, "d": d})
    return h_s, out
