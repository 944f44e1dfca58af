"""Served execution on the GPU: jobs arriving over time and running in one
continuously re-formed batch give bitwise the result each gives alone, and
every served result matches the oracle's run of the same job (within
1e-4 h, band membership exact away from the threshold)."""
import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import serve, synth

pytestmark = pytest.mark.gpu


def _requests(n, seed, steps_range=(20, 37)):
    rng = np.random.default_rng(seed)
    out = []
    for k, w in enumerate(synth.batch_jobs(n_jobs=n, seed=seed, n_range=(40, 64),
                                           pts_range=(2000, 8000))):
        w = dict(w)
        w["steps"] = int(rng.integers(*steps_range))
        w["arrival"] = 0.0005 * k
        w["interp"] = "weno"
        out.append(w)
    return out


def _alone(req, precision):
    from paper_2410_22205_amd import lsr
    job = lsr.Job(req["grid"], serve.job_params(req, precision), max_points=len(req["points"]))
    job.load_cloud(req["points"])
    job.init_phi(req["phi0"][0], req["phi0"][1])
    job.step(req["steps"], req["dt"], req["interp"])
    phi, band, _, si = job.extract()
    job.close()
    assert si == req["steps"]
    return phi.ravel(), band.ravel()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_served_results_equal_alone(precision):
    reqs = _requests(6, 4500)
    srv = serve.Server(max_active=8, group_steps=7, precision=precision)
    out = srv.run(reqs, keep_results=True)
    assert out["jobs"] == len(reqs) and not out["rejected"]
    assert out["max_batch"] >= 2  # the jobs did share the batch
    worst = 0.0
    for i, req in enumerate(reqs):
        phi, band = _alone(req, precision)
        np.testing.assert_array_equal(out["results"][i][0], phi)
        np.testing.assert_array_equal(out["results"][i][1], band)
        worst = max(worst, _against_oracle(req, out["results"][i][0], out["results"][i][1]))
    print(f"served {precision}: max |phi - oracle| {worst:.2e} h over {len(reqs)} jobs")


def test_shortest_first_parks_and_results_equal_alone():
    """The shortest-remaining-work policy sets running jobs aside for shorter
    arrivals and later resumes them (their state stays on the device): every
    result is still bitwise the job's result alone."""
    reqs = _requests(5, 4600, steps_range=(20, 25))
    reqs[0]["steps"] = 1000  # a long job first, shorter ones arriving while it runs
    for k, r in enumerate(reqs):
        r["arrival"] = 0.0 if k == 0 else 0.002 + 0.001 * k
    srv = serve.Server(max_active=8, group_steps=5, precision="fp32", policy="shortest",
                       short_budget=1, max_wait_s=0.03)
    out = srv.run(reqs, keep_results=True)
    assert out["jobs"] == len(reqs) and not out["rejected"]
    assert out["parked"] >= 1, out["parked"]
    for i, req in enumerate(reqs):
        phi, band = _alone(req, "fp32")
        np.testing.assert_array_equal(out["results"][i][0], phi)
        np.testing.assert_array_equal(out["results"][i][1], band)


def _against_oracle(req, phi, band):
    """The oracle's run of the request: its grid, cloud, phi0, dt, steps and
    interpolator; returns max |phi - oracle| in units of h."""
    g = req["grid"]
    h = g["h"]
    prm = oracle.default_params(g["dim"], h, gamma=req["gamma"], beta=req["beta"],
                                reinit_every=req["reinit_every"])
    d = oracle.distance(req["points"], g)
    phi0 = oracle.init_phi(g, req["phi0"][0], req["phi0"][1], prm["gamma"])
    ophi, _ = oracle.run(phi0, d, g, prm, req["dt"], req["interp"], req["steps"])
    ophi = ophi.ravel()
    err = float(np.abs(phi.astype(np.float64) - ophi).max())
    assert err <= 1e-4 * h, err / h
    np.testing.assert_array_equal(band, (np.abs(phi) < phi.dtype.type(prm["gamma"])).astype(np.uint8))
    sure = np.abs(np.abs(ophi) - prm["gamma"]) > 1e-6 * h
    assert not ((band.astype(bool) != (np.abs(ophi) < prm["gamma"])) & sure).any()
    return err / h


def test_budget_bounds_the_mix_and_sequential_replay_agrees():
    reqs = _requests(5, 4600)
    one = max(serve.footprint_bytes(r, "fp32") for r in reqs)
    srv = serve.Server(budget_bytes=2 * one, max_active=8, group_steps=5, precision="fp32")
    out = srv.run(reqs, keep_results=True)
    assert out["jobs"] == 5 and out["max_batch"] <= 2
    seq = serve.run_sequential(reqs, precision="fp32", keep_results=True)
    for i in range(len(reqs)):
        np.testing.assert_array_equal(out["results"][i][0], seq["results"][i][0])
    assert out["latency_ms"]["p99"] >= out["latency_ms"]["p50"] > 0
