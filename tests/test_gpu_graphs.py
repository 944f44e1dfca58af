"""Step loops recorded as HIP graphs: a replayed graph runs the kernels,
arguments and order of the direct launches, so a job or a batch gives bitwise
the results of the same run with graphs switched off; the graphs really were
recorded and replayed (capture/replay counts).  Graphs need a stream other
than the null stream, so every job and batch here gets one."""
import numpy as np
import pytest

from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu


def _lsr():
    from paper_2410_22205_amd import lsr
    return lsr


def _job(lsr, w, precision, stream):
    prm = dict(gamma=w["gamma"], beta=w["beta"], reinit_every=w["reinit_every"],
               precision=precision)
    job = lsr.Job(w["grid"], prm, max_points=len(w["points"]), stream=stream)
    job.load_cloud(w["points"])
    return job


def _runs(w, precision, graphs, steps, repeats=2):
    import torch
    lsr = _lsr()
    job = _job(lsr, w, precision, torch.cuda.Stream())
    job.set_graphs(graphs)
    out = []
    for _ in range(repeats):
        job.init_phi(w["phi0"][0], w["phi0"][1])
        job.step(steps, w["dt"], w["interp"])
        phi, band, nb, si = job.extract()
        out.append((phi, band, nb, si, job.counters()))
    counts = job.graph_counts()
    job.close()
    return out, counts


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_torus_steps_through_graphs_equal_direct(precision):
    # chunks of 2 x 10 steps: the first run launches its first chunk
    # directly, records the second and replays the third; the second run
    # replays all three; 5 steps at the end of each run stay direct
    w = synth.workload("torus3d", n=48, steps=65)
    direct, c0 = _runs(w, precision, False, 65)
    graph, c1 = _runs(w, precision, True, 65)
    assert c0 == (0, 0)
    assert c1 == (1, 4), (c1, _lsr().lsr_last_error())
    for (p0, b0, n0, s0, k0), (p1, b1, n1, s1, k1) in zip(direct, graph):
        np.testing.assert_array_equal(p1, p0)
        np.testing.assert_array_equal(b1, b0)
        assert (n1, s1) == (n0, s0) and s1 == 65
        assert k1 == k0
    # both runs of one job from the same initial data agree
    np.testing.assert_array_equal(graph[0][0], graph[1][0])


def test_circle_2d_steps_through_graphs_equal_direct():
    # 2D reinitialises every step: chunks of 2 steps
    w = synth.workload("circle2d", n=96, steps=9)
    direct, _ = _runs(w, "fp32", False, 9)
    graph, c1 = _runs(w, "fp32", True, 9)
    assert c1 == (1, 6), (c1, _lsr().lsr_last_error())
    for a, b in zip(direct, graph):
        np.testing.assert_array_equal(b[0], a[0])
        np.testing.assert_array_equal(b[1], a[1])
        assert b[4] == a[4]


def test_kernel_timing_launches_directly():
    """While kernel timing is on, step loops launch directly (no graph is
    recorded or replayed) and every step kernel is timed; with timing off
    the graphs come back, and the results are the same either way."""
    import torch
    lsr = _lsr()
    w = synth.workload("torus3d", n=64, steps=60)
    job = _job(lsr, w, "fp32", torch.cuda.Stream())
    lsr.lsr_profile_enable(job.handle, True, 100)
    job.init_phi(w["phi0"][0], w["phi0"][1])
    job.step(60, w["dt"], w["interp"])
    ms, n = lsr.lsr_profile_read(job.handle)
    timed = job.extract()[0]
    assert n == 60 and 0 < ms / n < 10.0
    assert job.graph_counts() == (0, 0)
    lsr.lsr_profile_enable(job.handle, False)
    job.init_phi(w["phi0"][0], w["phi0"][1])
    job.step(60, w["dt"], w["interp"])
    assert job.graph_counts() == (1, 1)  # chunks: direct, recorded, replayed
    np.testing.assert_array_equal(job.extract()[0], timed)
    job.close()


def test_batch_groups_through_graphs_equal_direct():
    import torch
    lsr = _lsr()
    ws = list(synth.batch_jobs(n_jobs=3, seed=4600, n_range=(40, 64),
                               pts_range=(2000, 8000), steps=40))
    res = {}
    for graphs in (False, True):
        batch = lsr.Batch(max_jobs=3, group_steps=10, stream=torch.cuda.Stream())
        batch.set_graphs(graphs)
        jobs = []
        for w in ws:
            j = _job(lsr, w, "fp32", torch.cuda.Stream())
            j.init_phi(w["phi0"][0], w["phi0"][1])
            batch.add(j, w["dt"], w["interp"])
            jobs.append(j)
        batch.step(40)
        res[graphs] = [(j.extract(), j.counters()) for j in jobs]
        counts = batch.graph_counts()
        if graphs:
            # every group has the same launch sequence: 1 direct, 1 recorded,
            # 2 replayed
            assert counts == (1, 2), counts
        else:
            assert counts == (0, 0)
        batch.close()
        for j in jobs:
            j.close()
    for ((p0, b0, n0, s0), k0), ((p1, b1, n1, s1), k1) in zip(res[False], res[True]):
        np.testing.assert_array_equal(p1, p0)
        np.testing.assert_array_equal(b1, b0)
        assert (n1, s1, k1) == (n0, s0, k0)


def test_batch_graphs_across_membership_changes():
    """Jobs join and leave between groups while recorded groups replay: each
    job still ends bitwise where it ends alone."""
    import torch
    lsr = _lsr()
    ws = list(synth.batch_jobs(n_jobs=3, seed=4700, n_range=(40, 56),
                               pts_range=(2000, 6000), steps=60))
    solo = []
    for w in ws:
        j = _job(lsr, w, "fp32", torch.cuda.Stream())
        j.set_graphs(False)
        j.init_phi(w["phi0"][0], w["phi0"][1])
        j.step(60, w["dt"], w["interp"])
        solo.append(j.extract()[0])
        j.close()
    batch = lsr.Batch(max_jobs=3, group_steps=10, stream=torch.cuda.Stream())
    jobs = []
    for w in ws:
        j = _job(lsr, w, "fp32", torch.cuda.Stream())
        j.init_phi(w["phi0"][0], w["phi0"][1])
        jobs.append(j)
    batch.add(jobs[0], ws[0]["dt"], ws[0]["interp"])
    batch.add(jobs[1], ws[1]["dt"], ws[1]["interp"])
    batch.step(30)                      # {0, 1}: direct, recorded, replayed
    jobs[2].step(30, ws[2]["dt"], ws[2]["interp"])
    batch.add(jobs[2], ws[2]["dt"], ws[2]["interp"])
    batch.step(20)                      # {0, 1, 2}: direct, recorded
    batch.remove(jobs[0])
    jobs[0].step(10, ws[0]["dt"], ws[0]["interp"])
    batch.step(10)                      # {1, 2}: the launch sequence of {0, 1}
    captured, replayed = batch.graph_counts()
    assert (captured, replayed) == (2, 2), (captured, replayed)
    batch.close()
    for k, j in enumerate(jobs):
        phi, band, nb, si = j.extract()
        assert si == 60
        np.testing.assert_array_equal(phi, solo[k])
        j.close()
