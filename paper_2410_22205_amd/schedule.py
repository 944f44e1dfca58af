"""The coarse-to-fine schedule of Section 4 on the GPU: Algorithm 1 run
several times on finer and finer grids.

Run r takes p and delta from Table param and dx, dt from eq. (dxdt)
(``lsr_schedule_run``); the first run starts from phi0 computed from the
cloud with gamma_S = K_S h_S (Section 3.6, ``lsr_init_phi_cloud``), every
later one from the previous run's steady state interpolated onto its grid
(``lsr_init_phi_resample``); each run steps until the energy test of eq.
(deltaEn) stops it (``lsr_run_to_steady``).  Every computation runs in the
library's kernels; this module only sequences the calls and owns the jobs.
"""
import numpy as np

from . import lsr

SPACING_CELLS = 64  # cells along the longest axis of the grid that bins the cloud for h_S


def cloud_box(points):
    pts = np.asarray(points, dtype=np.float64)
    return pts.min(axis=0), pts.max(axis=0)


def cloud_spacing(points, sample, precision="fp64", stream=None):
    """h_S of the cloud (Section 4) over the sampled point indices: the cloud
    is binned on a coarse grid around its box (the value does not depend on
    that grid)."""
    pts = np.asarray(points, dtype=np.float64)
    dim = pts.shape[1]
    lo, hi = cloud_box(pts)
    ext = float(max(hi - lo)) or 1.0
    h = ext / SPACING_CELLS
    n = tuple(int(np.ceil((hi[a] - lo[a]) / h)) + 5 for a in range(dim))
    grid = {"dim": dim, "n": n, "lo": tuple(float(lo[a] - 2 * h) for a in range(dim)), "h": h}
    job = lsr.Job(grid, {"precision": precision}, max_points=len(pts), stream=stream)
    try:
        job.load_cloud(pts)
        return job.cloud_spacing(sample)
    finally:
        job.close()


def grid_dict(g):
    dim = int(g.dim)
    return {"dim": dim, "n": tuple(int(g.n[a]) for a in range(dim)),
            "lo": tuple(float(g.lo[a]) for a in range(dim)), "h": float(g.h)}


def reconstruct(points, sample, interp, runs=3, K_S=2.0, precision="fp64", min_steps=10,
                max_steps=100, tol=1e-4, stream=None, keep_phi=True):
    """Runs 1..runs of the schedule.  Returns (h_S, [per run: grid, params
    (p, delta), dt, steps, energies, phi (host array, when keep_phi)])."""
    pts = np.asarray(points, dtype=np.float64)
    dim = pts.shape[1]
    lo, hi = cloud_box(pts)
    h_s = cloud_spacing(pts, sample, precision, stream)
    out = []
    prev = None
    try:
        for r in range(1, runs + 1):
            g, p, dt = lsr.lsr_schedule_run(r, dim, lo, hi, h_s, K_S)
            grid = grid_dict(g)
            prm = {f[0]: getattr(p, f[0]) for f in lsr.LsrParams._fields_}
            prm["precision"] = {"fp32": lsr.LSR_FP32, "fp64": lsr.LSR_FP64}[precision]
            job = lsr.Job(grid, prm, max_points=len(pts), stream=stream)
            job.load_cloud(pts)
            if prev is None:
                job.init_phi_cloud(K_S * h_s)
            else:
                job.init_phi_resample(prev, interp)
            steps, energies = job.run_to_steady(dt, interp, min_steps, max_steps, tol)
            rec = {"grid": grid, "p": prm["p"], "delta": prm["delta"], "dt": dt, "steps": steps,
                   "energies": energies}
            if keep_phi:
                rec["phi"] = job.extract()[0]
            out.append(rec)
            if prev is not None:
                prev.close()
            prev = job
    finally:
        if prev is not None:
            prev.close()
    return h_s, out
