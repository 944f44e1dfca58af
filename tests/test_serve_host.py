"""Host logic of the served loop: admission by byte budget (no GPU)."""
import numpy as np
import pytest

from paper_2410_22205_amd import serve, synth


def test_admission_is_first_come_first_served_within_budget():
    a = serve.Admission(budget_bytes=100, max_active=8)
    for key, nbytes in [("a", 40), ("b", 50), ("c", 30), ("d", 5)]:
        assert a.offer(key, nbytes)
    assert a.admit() == ["a", "b"]          # c does not fit; d may not overtake it
    assert a.used == 90 and list(a.queue) == [("c", 30), ("d", 5)]
    a.release("a")
    assert a.admit() == ["c", "d"] and a.used == 85
    a.release("b"), a.release("c"), a.release("d")
    assert a.used == 0 and not a.holding


def test_admission_caps_the_number_of_jobs():
    a = serve.Admission(budget_bytes=10 ** 9, max_active=2)
    for k in range(5):
        a.offer(k, 1)
    assert a.admit() == [0, 1]
    assert a.admit() == []
    a.release(1)
    assert a.admit() == [2]


def test_oversized_request_is_rejected_not_queued():
    a = serve.Admission(budget_bytes=100, max_active=4)
    assert not a.offer("big", 101)
    assert a.rejected == ["big"] and not a.queue
    with pytest.raises(ValueError):
        serve.Admission(budget_bytes=0, max_active=1)


def test_footprint_grows_with_grid_and_cloud():
    w = synth.batch_jobs(n_jobs=1, seed=4000, n_range=(64, 64), pts_range=(5000, 5000))[0]
    small = serve.footprint_bytes(w, "fp32")
    big_cloud = dict(w, points=w["points"].repeat(4, axis=0))
    assert serve.footprint_bytes(big_cloud, "fp32") > small
    assert serve.footprint_bytes(w, "fp64") > small
    n = 64 ** 3
    assert small > (2 * 4 + 16 + 8 + 12) * n  # phi x2, (grad d, d), d, lists


def test_served_stream_recipe():
    specs = synth.served_jobs(n_jobs=30)
    arr = [s["arrival"] for s in specs]
    assert arr == sorted(arr) and 0.5 < 30 / arr[-1] / 20.0 < 2.0
    for s in specs:
        assert 64 <= s["grid"]["n"][0] <= 320 and 200 <= s["steps"] <= 400
    reqs = serve.materialise(specs[:2])
    assert reqs[0]["points"].shape[1] == 3


def test_admission_limit_and_band_estimate():
    a = serve.Admission(budget_bytes=100, max_active=8)
    for k in range(4):
        a.offer(k, 10)
    assert a.admit(limit=1) == [0] and a.admit(limit=2) == [1, 2]
    g = synth.cube_grid(3, 101)
    req = {"grid": g, "gamma": 6 * g["h"], "phi0": ("sphere", (0.0, 0.0, 0.0, 0.5))}
    est = serve.band_estimate(req)
    from oracle import node_coords  # brute count of the shell
    r = np.linalg.norm(node_coords(g), axis=1)
    exact = int((np.abs(r - 0.5) < 6 * g["h"]).sum())
    assert abs(est - exact) < 0.02 * exact


def test_least_work_first_orders_by_remaining_work_within_the_budget():
    rem = {0: 900, 1: 30, 2: 50, 3: 10}
    work = {0: 300, 1: 10, 2: 20, 3: 5}
    # the three shortest fit 40 node updates per step; the long job waits
    assert serve.least_work_first([0, 1, 2, 3], rem, work, set(), 40) == [3, 1, 2]
    # a budget smaller than any job still runs the shortest one
    assert serve.least_work_first([0, 1, 2, 3], rem, work, set(), 1) == [3]
    # equal remaining work: the lower key first
    assert serve.least_work_first([5, 4], {4: 7, 5: 7}, {4: 1, 5: 1}, set(), 1) == [4]


def test_least_work_first_keeps_jobs_that_waited_too_long():
    rem = {0: 900, 1: 30, 2: 50}
    work = {0: 300, 1: 10, 2: 20}
    # the long job has waited too long: it runs, and the budget still admits
    # the shortest of the others
    assert serve.least_work_first([0, 1, 2], rem, work, {0}, 15) == [0, 1]
    assert serve.least_work_first([], {}, {}, set(), 10) == []
