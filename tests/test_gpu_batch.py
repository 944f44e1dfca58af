"""Batched execution: several independent jobs stepped by one launch per
kernel give bitwise the results of each job run alone (same launch shape),
whatever the mix of grids, interpolators and reinitialisation phases, and
when jobs join or leave between steps.  The solo runs are themselves checked
against the oracle by test_gpu_parity.py; one batched job is checked against
the oracle here as well."""
import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu


def _lsr():
    from paper_2410_22205_amd import lsr
    return lsr


def _jobs(precision, n=5, seed=4000, small=True):
    """Uneven grids, Q1/WENO alternating, random shape unions."""
    out = []
    for w in synth.batch_jobs(n_jobs=n, seed=seed, n_range=(40, 72) if small else (64, 192),
                              pts_range=(2000, 20000), steps=12):
        w["precision"] = precision
        out.append(w)
    return out


def _make(lsr, w, step0=0, lanes=None):
    h = w["grid"]["h"]
    prm = dict(gamma=w["gamma"], beta=w["beta"], reinit_every=w["reinit_every"],
               precision=w["precision"], p=w.get("p", 1.0))
    job = lsr.Job(w["grid"], prm, max_points=len(w["points"]))
    if lanes:
        job.set_launch(lanes)
    job.load_cloud(w["points"])
    job.init_phi(w["phi0"][0], w["phi0"][1], step0=step0)
    return job


def _solo(w, steps, step0=0, lanes=None):
    lsr = _lsr()
    job = _make(lsr, w, step0, lanes)
    job.step(steps, w["dt"], w["interp"])
    phi, band, nb, si = job.extract()
    cnt = job.counters()
    job.close()
    return phi, band, nb, si, cnt


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_solo_bitwise(precision):
    lsr = _lsr()
    ws = _jobs(precision)
    steps = 23  # crosses two reinitialisations
    solo = [_solo(w, steps) for w in ws]
    batch = lsr.Batch(max_jobs=len(ws), group_steps=8)
    jobs = [_make(lsr, w) for w in ws]
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    batch.step(steps)
    for (phi0, band0, nb0, si0, cnt0), j in zip(solo, jobs):
        phi, band, nb, si = j.extract()
        np.testing.assert_array_equal(phi, phi0)
        np.testing.assert_array_equal(band, band0)
        assert nb == nb0 and si == si0 == steps
        assert j.counters() == cnt0
    batch.close()
    for j in jobs:
        j.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_with_p2_members_equals_solo_bitwise(precision):
    """p = 2 members get their own energy launch before each batched step;
    mixed with p = 1 members they still match their solo runs bit for bit."""
    lsr = _lsr()
    ws = _jobs(precision, n=4, seed=4200)
    for k, w in enumerate(ws):
        w["p"] = 2.0 if k % 2 == 0 else 1.0
    steps = 13  # crosses a reinitialisation
    solo = [_solo(w, steps) for w in ws]
    batch = lsr.Batch(max_jobs=len(ws), group_steps=5)
    jobs = [_make(lsr, w) for w in ws]
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    batch.step(steps)
    for (phi0, band0, nb0, si0, cnt0), j in zip(solo, jobs):
        phi, band, nb, si = j.extract()
        np.testing.assert_array_equal(phi, phi0)
        np.testing.assert_array_equal(band, band0)
        assert nb == nb0 and si == si0 == steps
    batch.close()
    for j in jobs:
        j.close()


def test_p2_member_replaced_while_graphs_replay():
    """A p = 2 member leaves after the batch has recorded and replayed its
    groups, is destroyed, and a new p = 2 job of the same shape (whose
    workspace may reuse the old one's memory) joins: the energy launches key
    on the buffers they read, and every job still ends bitwise where it ends
    alone."""
    lsr = _lsr()
    ws = _jobs("fp32", n=2, seed=4300)
    for w in ws:
        w["p"] = 2.0
    solo_c = _solo(ws[0], 40)
    solo_b = _solo(ws[1], 100)
    # groups of 10 steps, one reinitialisation each: two alternating launch
    # sequences, recorded at their second sight and replayed from the fifth
    # group on
    import torch
    # a stream of its own: the null stream cannot be captured into graphs
    batch = lsr.Batch(max_jobs=2, group_steps=10, stream=torch.cuda.Stream())
    a, b = _make(lsr, ws[0]), _make(lsr, ws[1])
    batch.add(a, ws[0]["dt"], ws[0]["interp"])
    batch.add(b, ws[1]["dt"], ws[1]["interp"])
    batch.step(60)
    captured, replayed = batch.graph_counts()
    assert captured >= 2 and replayed >= 2, (captured, replayed)
    batch.remove(a)
    a.close()
    del a
    c = _make(lsr, ws[0])
    batch.add(c, ws[0]["dt"], ws[0]["interp"])
    batch.step(40)
    for (phi0, band0, nb0, si0, _), j in ((solo_c, c), (solo_b, b)):
        phi, band, nb, si = j.extract()
        np.testing.assert_array_equal(phi, phi0)
        np.testing.assert_array_equal(band, band0)
        assert nb == nb0 and si == si0
    batch.close()
    b.close()
    c.close()


def test_batch_with_mixed_phases_and_membership():
    lsr = _lsr()
    ws = _jobs("fp32", n=4, seed=4100)
    # job k starts at global step k (its own reinitialisation phase)
    solo = [_solo(w, 17, step0=k) for k, w in enumerate(ws)]
    batch = lsr.Batch(max_jobs=4, group_steps=5)
    jobs = [_make(lsr, w, step0=k) for k, w in enumerate(ws)]
    # jobs 0, 1 in the batch throughout; job 2 steps 4 alone, then joins;
    # job 3 steps 6 in the batch, leaves and finishes alone (17 steps each)
    batch.add(jobs[0], ws[0]["dt"], ws[0]["interp"])
    batch.add(jobs[1], ws[1]["dt"], ws[1]["interp"])
    batch.add(jobs[3], ws[3]["dt"], ws[3]["interp"])
    jobs[2].step(4, ws[2]["dt"], ws[2]["interp"])
    batch.step(4)
    batch.add(jobs[2], ws[2]["dt"], ws[2]["interp"])
    batch.step(2)
    batch.remove(jobs[3])
    jobs[3].step(11, ws[3]["dt"], ws[3]["interp"])
    batch.step(11)
    batch.close()
    for k, j in enumerate(jobs):
        phi, band, nb, si = j.extract()
        np.testing.assert_array_equal(phi, solo[k][0])
        assert si == 17 + k
        j.close()


def test_tuning_changes_speed_not_results():
    lsr = _lsr()
    ws = _jobs("fp32", n=3, seed=4200)
    solo = [_solo(w, 11, lanes=1) for w in ws]
    batch = lsr.Batch(max_jobs=3, group_steps=16)
    jobs = [_make(lsr, w) for w in ws]
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    lanes, bpc, ms = batch.tune()
    assert lanes in (1, 4) and bpc in (2, 4, 8) and ms > 0
    batch.step(11)
    for (phi0, *_), j in zip(solo, jobs):
        np.testing.assert_array_equal(j.extract()[0], phi0)
    batch.close()
    for j in jobs:
        j.close()


def test_batched_job_matches_oracle():
    lsr = _lsr()
    ws = _jobs("fp64", n=2, seed=4300)
    batch = lsr.Batch(max_jobs=2, group_steps=32)
    jobs = [_make(lsr, w) for w in ws]
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    batch.step(12)
    for w, j in zip(ws, jobs):
        g = w["grid"]
        prm = oracle.default_params(3, g["h"], gamma=w["gamma"], beta=w["beta"],
                                    reinit_every=w["reinit_every"])
        d = oracle.distance(w["points"], g)
        phi0 = oracle.init_phi(g, w["phi0"][0], w["phi0"][1], prm["gamma"])
        ophi, _ = oracle.run(phi0, d, g, prm, w["dt"], w["interp"], 12)
        phi = j.extract()[0]
        assert np.abs(phi - ophi).max() <= 1e-4 * g["h"]
    batch.close()
    for j in jobs:
        j.close()


def test_batch_rules():
    lsr = _lsr()
    w3 = _jobs("fp32", n=1, seed=4400)[0]
    w2 = synth.workload("circle2d", n=40, steps=3)
    w2["precision"] = "fp32"
    batch = lsr.Batch(max_jobs=2, group_steps=4)
    j3 = _make(lsr, w3)
    j2 = _make(lsr, w2)
    batch.add(j3, w3["dt"], w3["interp"])
    with pytest.raises(lsr.LsrError) as e:
        batch.add(j2, w2["dt"], w2["interp"])
    assert e.value.status == lsr.LSR_E_UNSUPPORTED
    with pytest.raises(lsr.LsrError) as e:
        j3.step(1, w3["dt"], w3["interp"])
    assert e.value.status == lsr.LSR_E_STATE
    with pytest.raises(lsr.LsrError) as e:
        batch.add(j3, w3["dt"], w3["interp"])
    assert e.value.status == lsr.LSR_E_STATE
    batch.step(2)
    assert j3.extract()[3] == 2
    batch.close()
    j3.step(1, w3["dt"], w3["interp"])
    assert j3.extract()[3] == 3
    j3.close()
    j2.close()


def test_tuned_shape_is_kept_for_the_same_signature():
    """A second batch of the same dimension, precision, interpolator mix and
    size gets the first one's tuned shape without timing again (the same
    time comes back)."""
    lsr = _lsr()
    ws = _jobs("fp32", n=2, seed=4800)
    out = []
    for _ in range(2):
        batch = lsr.Batch(max_jobs=2, group_steps=4)
        jobs = [_make(lsr, w) for w in ws]
        for w, j in zip(ws, jobs):
            batch.add(j, w["dt"], w["interp"])
        out.append(batch.tune())
        batch.close()
        for j in jobs:
            j.close()
    assert out[0] == out[1] and out[0][2] > 0


@pytest.mark.parametrize("streams", [2, 1])
def test_cache_groups_on_two_streams(streams):
    """Jobs too large to share the device's last-level cache are stepped in
    separate cache groups; on two streams the groups overlap.  Every job
    still ends bitwise where it ends alone."""
    lsr = _lsr()
    ws = []
    for w in synth.batch_jobs(n_jobs=3, seed=4900, n_range=(168, 176), pts_range=(5000, 9000),
                              steps=12):
        w["precision"] = "fp32"
        ws.append(w)
    solo = [_solo(w, 12)[0] for w in ws]
    batch = lsr.Batch(max_jobs=3, group_steps=6)
    batch.set_streams(streams)
    jobs = [_make(lsr, w) for w in ws]
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    batch.step(12)
    for k, j in enumerate(jobs):
        np.testing.assert_array_equal(j.extract()[0], solo[k])
    batch.close()
    for j in jobs:
        j.close()


def test_tune_cache_file(tmp_path):
    """A tuned shape written to the cache file is found again: a batch whose
    signature has a line in the file takes that line's shape and time
    without timing, and a new signature's tuning appends its line."""
    lsr = _lsr()
    ws = _jobs("fp64", n=2, seed=4900)
    jobs = [_make(lsr, w) for w in ws]
    nodes = sum(int(np.prod(w["grid"]["n"])) for w in ws)
    p2 = 1
    while p2 < nodes:
        p2 *= 2
    nq = sum(w["interp"] == "q1" for w in ws)
    path = tmp_path / "tune.txt"
    path.write_text(f"3 1 {nq} {len(ws) - nq} {p2} 4 2 0.125\n")
    lsr.lsr_set_tune_cache(str(path))
    batch = lsr.Batch(max_jobs=2, group_steps=4)
    for w, j in zip(ws, jobs):
        batch.add(j, w["dt"], w["interp"])
    assert batch.tune() == (4, 2, 0.125)
    batch.close()
    for j in jobs:
        j.close()
    # a signature no other test tunes (one FP64 WENO job of 130^3 nodes):
    # timed, and its line appended
    w = dict(synth.workload("torus3d", n=130, steps=1), precision="fp64")
    job = _make(lsr, w)
    batch = lsr.Batch(max_jobs=1, group_steps=4)
    batch.add(job, w["dt"], w["interp"])
    lanes, bpc, ms = batch.tune()
    batch.close()
    job.close()
    lines = [ln for ln in path.read_text().split("\n") if ln.strip()]
    assert len(lines) == 2 and lines[1].startswith("3 1 0 1 4194304 ")
    assert lines[1].split()[5:7] == [str(lanes), str(bpc)] and ms > 0
    lsr.lsr_set_tune_cache(None)
