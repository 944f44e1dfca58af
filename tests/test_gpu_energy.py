"""GPU parity of the energy functional E_p (Section 3.5) through the C ABI:
lsr_energy on the device's phi and d against the oracle's E_p of the same
nodal values.  Both sum in double over the same cells with the same
arithmetic per cell (no FMA contraction) in different orders, and take the
same subcell decisions; tolerance 1e-12 relative."""
import math

import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _job(w, precision):
    from paper_2410_22205_amd import lsr
    g = w["grid"]
    prm = dict(gamma=w["gamma"], beta=w["beta"], reinit_every=w.get("reinit_every", 10),
               precision=precision)
    return lsr.Job(g, prm, max_points=len(w["points"]))


def _evolved(name, n, steps, precision):
    w = synth.workload(name, n=n)
    job = _job(w, precision)
    job.load_cloud(w["points"])
    job.init_phi(w["phi0"][0], w["phi0"][1])
    if steps:
        job.step(steps, w["dt"], w["interp"])
    return w, job


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,n,steps", [("circle2d", 128, 30), ("circle2d", 61, 5),
                                          ("torus3d", 48, 12), ("torus3d", 37, 3)])
@pytest.mark.parametrize("p", [1.0, 2.0])
def test_energy_matches_oracle(name, n, steps, precision, p):
    w, job = _evolved(name, n, steps, precision)
    try:
        phi, _, _, _ = job.extract()
        d = job.distance()
        e = job.energy(p)
        e3 = job.energy(p, R=3) if w["grid"]["dim"] == 3 else None
    finally:
        job.close()
    eo = oracle.energy(phi.astype(np.float64), d, w["grid"], p)
    assert eo > 0
    assert abs(e - eo) <= TOL * eo, (e, eo)
    if e3 is not None:
        eo3 = oracle.energy(phi.astype(np.float64), d, w["grid"], p, R=3)
        assert abs(e3 - eo3) <= TOL * eo3, (e3, eo3)


def test_energy_circle_of_64_points():
    """The unit circle's signed distance and the 64-point cloud on it: E_2
    close to the exact 7.1035e-2 and equal to the oracle's."""
    from paper_2410_22205_amd import lsr
    g = synth.cube_grid(2, 801, -1.5, 1.5)
    th = 2.0 * np.pi * np.arange(64) / 64.0
    pts = np.stack([np.cos(th), np.sin(th)], 1)
    X = oracle.node_coords(g)
    phi = (np.linalg.norm(X, axis=1) - 1.0).reshape(g["n"])
    job = lsr.Job(g, dict(gamma=6 * g["h"], beta=3 * g["h"], precision="fp64"), max_points=64)
    try:
        job.load_cloud(pts)
        job.init_phi(phi0=phi)
        cut, _, _, _ = job.extract()
        d = job.distance()
        e = job.energy(2.0)
    finally:
        job.close()
    exact = math.sqrt(256.0 * (math.pi / 64.0 - math.sin(math.pi / 64.0)))
    assert abs(e - exact) / exact < 5e-3
    eo = oracle.energy(cut, d, g, 2.0)
    assert abs(e - eo) <= TOL * eo


def _planted(dim, plant):
    """A sphere's (circle's) signed distance with a planted second front far
    from it, where the cut holds phi at +gamma:
      split - a 2^dim block of nodes at -gamma: front cells none of whose
              vertices is on the band;
      mate  - one node at -gamma whose 3^dim neighbourhood is at +gamma/2, on
              the band: front cells whose lower corner is off the band."""
    from paper_2410_22205_amd import lsr
    n = 40 if dim == 3 else 81
    g = synth.cube_grid(dim, n, -1.5, 1.5)
    h = g["h"]
    gamma = 6 * h
    rng = np.random.default_rng(11)
    m = 400 if dim == 3 else 64
    v = rng.normal(size=(m, dim))
    pts = 0.6 * v / np.linalg.norm(v, axis=1, keepdims=True)
    X = oracle.node_coords(g)
    phi = (np.linalg.norm(X, axis=1) - 0.6).reshape(g["n"])
    clean = phi.copy()
    c = (5,) * dim
    if plant == "split":
        phi[tuple(slice(q, q + 2) for q in c)] = -1.0
    else:
        phi[tuple(slice(q - 1, q + 2) for q in c)] = 0.5 * gamma
        phi[c] = -1.0
    job = lsr.Job(g, dict(gamma=gamma, beta=3 * h, precision="fp64"), max_points=m)
    job.load_cloud(pts)
    job.init_phi(phi0=phi)
    return g, gamma, clean, job


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("plant", ["split", "mate"])
def test_energy_front_off_the_band(dim, plant):
    """Every front cell of the grid counts, also those away from the band:
    equal to the oracle's sum, which without the planted cells would be
    another one."""
    g, gamma, clean, job = _planted(dim, plant)
    try:
        cut, _, _, _ = job.extract()
        d = job.distance()
        e = job.energy(2.0)
    finally:
        job.close()
    eo = oracle.energy(cut, d, g, 2.0)
    assert abs(e - eo) <= TOL * eo, (e, eo)
    e_clean = oracle.energy(np.clip(clean, -gamma, gamma), d, g, 2.0)
    assert abs(eo - e_clean) > 1e-6 * eo


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_without_front_is_zero(dim):
    """phi0 a sphere that holds the whole grid: no cell is crossed."""
    w = synth.workload("circle2d" if dim == 2 else "torus3d", n=32)
    job = _job(w, "fp64")
    try:
        job.load_cloud(w["points"])
        job.init_phi("sphere", (0.0, 0.0, 0.0, 5.0))
        assert job.energy(2.0) == 0.0
    finally:
        job.close()


def test_energy_arguments():
    from paper_2410_22205_amd import lsr
    w = synth.workload("circle2d", n=32)
    job = _job(w, "fp32")
    try:
        with pytest.raises(RuntimeError):
            job.energy(2.0)  # no phi, no d yet
        job.load_cloud(w["points"])
        job.init_phi(w["phi0"][0], w["phi0"][1])
        for bad in (0.0, -1.0, float("nan")):
            with pytest.raises(RuntimeError):
                job.energy(bad)
        with pytest.raises(RuntimeError):
            lsr.lsr_energy(job.handle, 2.0, 0)
        assert job.energy(1.0) > 0
    finally:
        job.close()


# ------------------------------------------------ the p = 2 loop (Section 2)

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,n,steps", [("circle2d", 128, 25), ("torus3d", 40, 12)])
def test_p2_run_matches_oracle(name, n, steps, precision):
    """p = 2: every step computes E_2 of the current phi on the device and
    scales C by d / E_2 (Algorithm 1, step 2); the run follows the oracle's
    loop with the energy step within 1e-4 h, band exact away from gamma."""
    from test_gpu_parity import check_band, check_phi, gpu_run, oracle_params
    w = synth.workload(name, n=n)
    extra = {"p": 2.0}
    phi, band, _, _, cnt, _ = gpu_run(w, steps=steps, extra=extra, precision=precision)
    g = w["grid"]
    prm = oracle_params(w, extra)
    d = oracle.distance(w["points"], g)
    phi0 = oracle.init_phi(g, w["phi0"][0], w["phi0"][1], prm["gamma"])
    ophi, energies = oracle.run_p(phi0, d, g, prm, w["dt"], w["interp"], steps)
    assert all(e > 0 for e in energies)
    check_phi(phi, ophi, g["h"], 1e-4)
    check_band(band, phi, ophi, prm["gamma"], g["h"])
    # the p = 1 run from the same start ends elsewhere: the energy factor acts
    phi1, _, _, _, _, _ = gpu_run(w, steps=steps, precision=precision)
    assert np.abs(phi1.astype(np.float64) - ophi).max() > 1e-3 * g["h"]


def test_p_other_than_1_or_2_is_refused():
    from paper_2410_22205_amd import lsr
    w = synth.workload("circle2d", n=32)
    with pytest.raises(RuntimeError):
        lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"], p=1.5), max_points=10)


@pytest.mark.parametrize("p", [1.0, 2.0])
def test_run_to_steady_follows_the_stopping_test(p):
    """lsr_run_to_steady stops where the oracle's test of eq. (deltaEn) does on
    the energies it reports, and the last of them is E_2 of the final phi."""
    from paper_2410_22205_amd import lsr
    w = synth.workload("circle2d", n=64)
    job = lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"], reinit_every=1, p=p,
                                  precision="fp64"), max_points=len(w["points"]))
    try:
        job.load_cloud(w["points"])
        job.init_phi(w["phi0"][0], w["phi0"][1])
        n, e = job.run_to_steady(w["dt"], w["interp"])
        last = job.energy(2.0)
    finally:
        job.close()
    assert 10 <= n <= 100 and len(e) == n + 1
    assert [oracle.stop_rule(e, m) for m in range(n + 1)] == [False] * n + [True]
    assert last == e[-1]
