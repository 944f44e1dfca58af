"""Seeded synthetic point clouds and workload descriptions.

This module is the only code that both the HIP path and the CPU oracle see:
it draws point clouds and states grids and parameters, and holds none of the
reconstruction method's arithmetic.  Everything is NumPy with PCG64 streams
(``numpy.random.default_rng(seed)``), so a (generator, seed) pair always
gives the same cloud.

The shapes follow the paper's test families (Section 4: circle in 2D, sphere,
composite solids and scanned objects in 3D).  The scanned clouds are not
available; ``union_cloud`` stands in for them with their salient features
(non-uniform density, holes, two bodies).
"""
import math

import numpy as np

# ------------------------------------------------------------------ clouds


def circle_cloud(n, radius, seed, centre=(0.0, 0.0)):
    """n points on a circle at uniformly drawn angles."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return np.stack([centre[0] + radius * np.cos(t), centre[1] + radius * np.sin(t)], axis=1)


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sphere_points(rng, n, radius, centre=(0.0, 0.0, 0.0)):
    return np.asarray(centre) + radius * _unit_vectors(rng, n)


def torus_points(rng, n, R, r):
    """Area-uniform points on a torus with axis z centred at the origin: the
    tube angle is drawn by rejection with acceptance (R + r cos v)/(R + r)."""
    out = np.empty((0, 3))
    while len(out) < n:
        m = 2 * (n - len(out)) + 16
        u = rng.uniform(0.0, 2.0 * math.pi, size=m)
        v = rng.uniform(0.0, 2.0 * math.pi, size=m)
        keep = rng.uniform(size=m) < (R + r * np.cos(v)) / (R + r)
        u, v = u[keep], v[keep]
        ring = R + r * np.cos(v)
        pts = np.stack([ring * np.cos(u), ring * np.sin(u), r * np.sin(v)], axis=1)
        out = np.concatenate([out, pts])
    return out[:n]


def ellipsoid_points(rng, n, axes, centre=(0.0, 0.0, 0.0)):
    """Area-uniform points on an axis-aligned ellipsoid: a uniform direction is
    mapped onto the surface and accepted with probability proportional to the
    local area stretch."""
    a, b, c = axes
    out = np.empty((0, 3))
    top = max(b * c, a * c, a * b)
    while len(out) < n:
        m = 2 * (n - len(out)) + 16
        u = _unit_vectors(rng, m)
        stretch = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.uniform(size=m) < stretch / top
        out = np.concatenate([out, u[keep] * np.array([a, b, c])])
    return out[:n] + np.asarray(centre)


def torus_cloud(n, R, r, noise_sigma, seed):
    """Configuration of the 3D single-instance workload: area-uniform torus
    points plus isotropic Gaussian noise."""
    rng = np.random.default_rng(seed)
    pts = torus_points(rng, n, R, r)
    if noise_sigma > 0:
        pts = pts + rng.normal(scale=noise_sigma, size=pts.shape)
    return pts


def _ellipsoid_area(axes):
    # Knud Thomsen's approximation, p = 1.6075 (only used to mix components).
    a, b, c = axes
    p = 1.6075
    return 4.0 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1.0 / p)


def union_cloud(n, seed, sphere_c=(-0.3, 0.0, 0.0), sphere_r=0.4, ell_c=(0.3, 0.0, 0.0),
                ell_axes=(0.5, 0.3, 0.25), ramp=(0.1, 1.0), hole_r=0.1, n_holes=2):
    """Boundary of the union of a sphere and an ellipsoid, sampled with a
    density that ramps linearly by a factor ramp[1]/ramp[0] along a seeded
    direction, with n_holes seeded cap-shaped holes of radius hole_r."""
    rng = np.random.default_rng(seed)
    sc, ec = np.asarray(sphere_c), np.asarray(ell_c)
    ea = np.asarray(ell_axes)
    direction = _unit_vectors(rng, 1)[0]
    a_s = 4.0 * math.pi * sphere_r ** 2
    a_e = _ellipsoid_area(ell_axes)

    def raw(m):
        k = rng.uniform(size=m) < a_s / (a_s + a_e)
        ps = sphere_points(rng, int(k.sum()), sphere_r, sc)
        pe = ellipsoid_points(rng, int((~k).sum()), ell_axes, ec)
        # keep only points on the union's boundary
        ps = ps[np.sum(((ps - ec) / ea) ** 2, axis=1) > 1.0]
        pe = pe[np.linalg.norm(pe - sc, axis=1) > sphere_r]
        return np.concatenate([ps, pe])

    pre = raw(100_000)
    proj = pre @ direction
    lo, hi = float(proj.min()), float(proj.max())
    holes = pre[rng.choice(len(pre), size=n_holes, replace=False)]
    out = np.empty((0, 3))
    while len(out) < n:
        cand = raw(2 * (n - len(out)) + 64)
        w = ramp[0] + (ramp[1] - ramp[0]) * (cand @ direction - lo) / (hi - lo)
        cand = cand[rng.uniform(size=len(cand)) < w]
        for hc in holes:
            cand = cand[np.linalg.norm(cand - hc, axis=1) > hole_r]
        out = np.concatenate([out, cand])
    return out[:n]


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def random_union_cloud(n, seed, noise_sigma=0.0, max_radius=0.6):
    """1-3 randomly placed and rotated spheres, tori or ellipsoids whose
    surfaces all lie within max_radius of the origin, sampled by area."""
    rng = np.random.default_rng(seed)
    while True:
        parts = []
        for _ in range(int(rng.integers(1, 4))):
            kind = int(rng.integers(0, 3))
            centre = _unit_vectors(rng, 1)[0] * 0.2 * rng.uniform() ** (1.0 / 3.0)
            rot = _rotation(rng)
            if kind == 0:
                r = rng.uniform(0.15, 0.35)
                parts.append(("sphere", centre, rot, (r,), 4 * math.pi * r * r))
            elif kind == 1:
                R, r = rng.uniform(0.25, 0.40), rng.uniform(0.10, 0.15)
                parts.append(("torus", centre, rot, (R, r), 4 * math.pi ** 2 * R * r))
            else:
                ax = tuple(rng.uniform(0.15, 0.35, size=3))
                parts.append(("ellipsoid", centre, rot, ax, _ellipsoid_area(ax)))
        area = np.array([p[4] for p in parts])
        counts = rng.multinomial(n, area / area.sum())
        pts = []
        for (kind, centre, rot, prm, _), m in zip(parts, counts):
            if kind == "sphere":
                local = sphere_points(rng, m, prm[0])
            elif kind == "torus":
                local = torus_points(rng, m, prm[0], prm[1])
            else:
                local = ellipsoid_points(rng, m, prm)
            pts.append(local @ rot.T + centre)
        pts = np.concatenate(pts)
        if np.linalg.norm(pts, axis=1).max() <= max_radius:
            break
    if noise_sigma > 0:
        pts = pts + rng.normal(scale=noise_sigma, size=pts.shape)
    return pts


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of a Poisson stream with the given mean rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# -------------------------------------------------------------- workloads


def cube_grid(dim, n, lo=-1.0, hi=1.0):
    """n nodes per axis on [lo, hi]^dim, h = (hi - lo)/(n - 1)."""
    return {"dim": dim, "n": (n,) * dim, "lo": (lo,) * dim, "h": (hi - lo) / (n - 1)}


def workload(name, n=None, steps=None):
    """Grid, cloud, initial data and run parameters of a named workload.

    circle2d  - 2D circle: 128^2 on [-1,1]^2, 200 points on r = 0.5, phi0 circle
                r = 0.9, Q1, dt = h, 200 steps, band 6h, reinit every step.
    torus3d   - 3D single instance: 128^3, 20k torus points (R 0.5, r 0.2)
                plus N(0, (0.2h)^2) noise, phi0 sphere r = 0.9, WENO, dt = h/2,
                300 steps, band 6h, reinit every 10 steps.
    union3d   - 3D non-uniform: 256^3, 200k points on a sphere/ellipsoid union
                with a 10x density ramp and two holes, phi0 sphere r = 0.9,
                WENO, dt = h/2, 400 steps, band 6h, reinit every 10 steps.
    ``n`` and ``steps`` override the grid size and step count (the same recipe
    at a smaller size, for tests).
    """
    if name == "circle2d":
        N = n or 128
        grid = cube_grid(2, N)
        h = grid["h"]
        return dict(name=name, grid=grid, points=circle_cloud(200, 0.5, seed=1),
                    phi0=("sphere", (0.0, 0.0, 0.0, 0.9)), interp="q1", dt=h,
                    steps=steps or 200, gamma=6 * h, beta=3 * h, reinit_every=1)
    if name == "torus3d":
        N = n or 128
        grid = cube_grid(3, N)
        h = grid["h"]
        return dict(name=name, grid=grid,
                    points=torus_cloud(20_000, 0.5, 0.2, 0.2 * h, seed=2),
                    phi0=("sphere", (0.0, 0.0, 0.0, 0.9)), interp="weno", dt=0.5 * h,
                    steps=steps or 300, gamma=6 * h, beta=3 * h, reinit_every=10)
    if name == "union3d":
        N = n or 256
        grid = cube_grid(3, N)
        h = grid["h"]
        return dict(name=name, grid=grid, points=union_cloud(200_000, seed=3),
                    phi0=("sphere", (0.0, 0.0, 0.0, 0.9)), interp="weno", dt=0.5 * h,
                    steps=steps or 400, gamma=6 * h, beta=3 * h, reinit_every=10)
    raise ValueError(f"unknown workload {name!r}")


def tie_free_radius(h):
    """Radius of the initial sphere of the multi-job workloads.  On a grid
    with rational spacing a rational radius puts some nodes (Pythagorean
    triples) at exactly |phi0| = gamma, where band membership is decided by
    the last bit of rounding and the two sides of a comparison may decide it
    differently; the reinitialisation then turns that into an O(h) change of
    the node's value.  An offset of (sqrt(2)/10) h keeps every |phi0| off the
    thresholds by far more than rounding."""
    return min(0.9, 1.0 - 9.0 * h) - 0.1 * math.sqrt(2.0) * h


def batch_jobs(n_jobs=64, seed=4000, n_range=(64, 192), pts_range=(5_000, 150_000), steps=200):
    """Independent jobs of the batched workload: grid size uniform in
    n_range, cloud size uniform in pts_range, random shape unions, Q1 and
    WENO alternating, phi0 a sphere of radius min(0.9, 1 - gamma - 3h)
    less an irrational fraction of h (see tie_free_radius)."""
    jobs = []
    for i in range(n_jobs):
        rng = np.random.default_rng(seed + i)
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        npts = int(rng.integers(pts_range[0], pts_range[1] + 1))
        grid = cube_grid(3, N)
        h = grid["h"]
        r0 = tie_free_radius(h)
        jobs.append(dict(name=f"job{i}", grid=grid, points=random_union_cloud(npts, seed + i),
                         phi0=("sphere", (0.0, 0.0, 0.0, r0)),
                         interp="q1" if i % 2 == 0 else "weno", dt=0.5 * h, steps=steps,
                         gamma=6 * h, beta=3 * h, reinit_every=10))
    return jobs


def served_jobs(n_jobs=400, seed=5, rate=20.0, n_range=(64, 320), pts_range=(5_000, 1_000_000),
                steps_range=(200, 400)):
    """Request stream of the served workload: Poisson arrivals, grid size
    uniform in n_range, log-uniform cloud size, noise sigma uniform in
    [0, h/2], WENO, step count uniform in steps_range."""
    arrivals = poisson_arrivals(n_jobs, rate, seed)
    jobs = []
    for i in range(n_jobs):
        rng = np.random.default_rng(seed * 100_000 + i)
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        npts = int(round(math.exp(rng.uniform(math.log(pts_range[0]), math.log(pts_range[1])))))
        grid = cube_grid(3, N)
        h = grid["h"]
        sigma = rng.uniform(0.0, 0.5 * h)
        r0 = tie_free_radius(h)
        jobs.append(dict(name=f"req{i}", arrival=float(arrivals[i]), grid=grid,
                         cloud=("random_union", npts, seed * 100_000 + i, sigma),
                         phi0=("sphere", (0.0, 0.0, 0.0, r0)), interp="weno", dt=0.5 * h,
                         steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
                         gamma=6 * h, beta=3 * h, reinit_every=10))
    return jobs


def make_cloud(spec):
    kind = spec[0]
    if kind == "random_union":
        _, npts, seed, sigma = spec
        return random_union_cloud(npts, seed, noise_sigma=sigma)
    raise ValueError(kind)
