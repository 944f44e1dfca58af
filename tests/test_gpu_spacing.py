"""GPU parity of the cloud resolution h_S (Section 4, the text after eq.
dxdt) through lsr_cloud_spacing: the same sampled indices give the oracle's
mean nearest-neighbour distance.  Every per-point distance is the exact
minimum in double on both sides; the means are summed in different orders:
tolerance 1e-12 relative."""
import math

import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu


def _spacing(grid, pts, sample, max_points=None):
    from paper_2410_22205_amd import lsr
    job = lsr.Job(grid, dict(gamma=6 * grid["h"], beta=3 * grid["h"]),
                  max_points=max_points or len(pts))
    try:
        job.load_cloud(pts)
        return job.cloud_spacing(sample)
    finally:
        job.close()


def test_circle_of_64_points():
    g = synth.cube_grid(2, 129, -1.5, 1.5)
    th = 2.0 * np.pi * np.arange(64) / 64.0
    pts = np.stack([np.cos(th), np.sin(th)], 1)
    sample = np.random.default_rng(3).choice(64, size=6, replace=False)
    h = _spacing(g, pts, sample)
    assert abs(h - 2.0 * math.sin(math.pi / 64.0)) < 1e-14
    assert h == pytest.approx(oracle.cloud_spacing(pts, sample), rel=1e-12)


@pytest.mark.parametrize("case", ["torus3d", "circle2d", "dense", "union3d"])
def test_spacing_matches_oracle(case):
    if case == "dense":  # many points per 4h bin: the cloud is sorted by the finer bins
        g = synth.cube_grid(3, 72)
        pts = synth.torus_cloud(80_000, 0.3, 0.1, 0.0, seed=21)
    else:
        w = synth.workload(case)
        g, pts = w["grid"], np.asarray(w["points"])
    n = len(pts)
    sample = np.random.default_rng(31).choice(n, size=max(1, n // 10), replace=False)
    h = _spacing(g, pts, sample)
    assert h > 0
    assert h == pytest.approx(oracle.cloud_spacing(pts, sample), rel=1e-12)


def test_duplicates_and_arguments():
    from paper_2410_22205_amd import lsr
    g = synth.cube_grid(3, 32)
    pts = synth.torus_cloud(3000, 0.5, 0.2, 0.0, seed=5)
    dup = np.vstack([pts, pts[:10]])
    sample = np.arange(0, 40)
    h = _spacing(g, dup, sample)
    assert h == pytest.approx(oracle.cloud_spacing(dup, sample), rel=1e-12)
    job = lsr.Job(g, dict(gamma=6 * g["h"], beta=3 * g["h"]), max_points=len(pts))
    try:
        with pytest.raises(RuntimeError):
            job.cloud_spacing([0])  # no cloud loaded
        job.load_cloud(pts)
        with pytest.raises(RuntimeError):
            job.cloud_spacing([0, len(pts)])  # an index outside the cloud
        assert job.cloud_spacing([1, 2, 3]) > 0  # usable after the refusal
        before = job.cloud_spacing([1, 2, 3])
        bad = pts.copy()
        bad[0, 0] = 5.0  # outside the grid's box: the load fails ...
        with pytest.raises(RuntimeError):
            job.load_cloud(bad)
        # ... and leaves the job as it was: the previous cloud is still there
        assert job.cloud_spacing([1, 2, 3]) == before
    finally:
        job.close()
