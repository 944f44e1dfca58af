"""Served reconstruction: jobs arrive over time, are admitted while their
device footprint fits an HBM budget, and run with continuous batching.

Life of a request:
  queued    arrived, waiting for memory (first come, first served)
  loading   workspace taken; cloud upload, distance field and phi0 enqueued on
            a side stream while the running jobs keep stepping
  ready     loaded, waiting for room in the per-step work budget (or set
            aside for jobs with less work left)
  running   member of the shared batch; stepped together with the others
  finishing left the batch at a step boundary; phi and the band copied out
  done      copy-out complete; latency = completion - arrival; memory freed

Two budgets: device bytes decide which requests may hold a workspace (and so
start loading early), and the band nodes updated per step decide which loaded
jobs step together.  By default the jobs with the least work left step first
(up to 1M band nodes per step while few requests wait, up to 8M when many
do): a short job does not wait at a long job's pace, and the long job, set
aside with its state on the device, resumes when the short ones are done or
when it has waited too long.

Every job's phi, d and band stay in its own device workspace for its whole
life; nothing goes to the host between steps.  The batch steps all members
the same number of steps per call, so each call runs to the next step at
which a member finishes (at most group_steps); jobs that are ready join at
those boundaries.

Results do not depend on the mix: the batched kernels evaluate each node
exactly as the single-job kernels do (see tests/test_gpu_serve.py).
"""
import collections
import time

import numpy as np

from . import lsr


def job_params(req, precision):
    return dict(gamma=req["gamma"], beta=req["beta"], reinit_every=req["reinit_every"],
                precision=precision)


def band_estimate(req):
    """Band nodes of the initial sphere: nodes within gamma of its surface."""
    g = req["grid"]
    h, gam = g["h"], req["gamma"]
    kind, args = req["phi0"]
    r = args[3] if kind == "sphere" else args[4]
    if g["dim"] == 3:
        vol = 4.0 / 3.0 * np.pi * ((r + gam) ** 3 - max(r - gam, 0.0) ** 3) / h ** 3
    else:
        vol = np.pi * ((r + gam) ** 2 - max(r - gam, 0.0) ** 2) / h ** 2
    return int(min(vol, np.prod(g["n"][: g["dim"]])))


def footprint_bytes(req, precision):
    """Device bytes a request holds while admitted: the job workspace (state,
    lists, binned cloud), the uploaded cloud, and the result buffers."""
    g = req["grid"]
    grid = lsr.make_grid(g)
    prm = lsr.lsr_params_default(grid.dim, grid.h)
    for k, v in job_params(req, precision).items():
        if k == "precision":
            v = lsr.LSR_FP64 if v == "fp64" else lsr.LSR_FP32
        setattr(prm, k, v)
    n_pts = len(req["points"])
    nodes = int(np.prod(g["n"][: g["dim"]]))
    e = 8 if precision == "fp64" else 4
    return (lsr.lsr_workspace_bytes(grid, prm, n_pts) + 8 * g["dim"] * n_pts
            + (e + 1) * nodes)


class Admission:
    """First-come first-served admission against a byte budget and a cap on
    the number of jobs holding device memory.  Pure host logic."""

    def __init__(self, budget_bytes, max_active):
        if budget_bytes <= 0 or max_active < 1:
            raise ValueError("need a positive budget and max_active >= 1")
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.used = 0
        self.holding = {}
        self.queue = collections.deque()
        self.rejected = []

    def offer(self, key, nbytes):
        """A request arrives.  One that could never fit is rejected at once."""
        if nbytes > self.budget:
            self.rejected.append(key)
            return False
        self.queue.append((key, int(nbytes)))
        return True

    def admit(self, limit=None):
        """Keys admitted now (at most limit), in arrival order.  The head of
        the queue waits until it fits; later requests do not overtake it."""
        out = []
        while self.queue and len(self.holding) < self.max_active and (limit is None
                                                                       or len(out) < limit):
            key, nbytes = self.queue[0]
            if self.used + nbytes > self.budget:
                break
            self.queue.popleft()
            self.holding[key] = nbytes
            self.used += nbytes
            out.append(key)
        return out

    def release(self, key):
        self.used -= self.holding.pop(key)


def least_work_first(cands, remaining, work, sticky, budget):
    """The jobs that run next under the "shortest" policy: every job in
    sticky, then the others in order of remaining work (ties by key) while
    their per-step work adds up to at most budget (the first always).
    Pure host logic."""
    keep = [i for i in cands if i in sticky]
    w_sum = 0
    for i in sorted((i for i in cands if i not in sticky), key=lambda i: (remaining[i], i)):
        if w_sum and w_sum + work[i] > budget:
            break
        keep.append(i)
        w_sum += work[i]
    return keep


class _Live:
    __slots__ = ("req", "job", "ev", "left", "phi", "band", "pts", "state")


def _percentiles(x):
    if not x:
        return {"p50": None, "p99": None}
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))}


class Server:
    """Continuous-batching server on the current device.

    budget_bytes: HBM the jobs may hold together (default: 80 % of the free
    device memory); max_active: jobs holding memory at once (also the batch
    capacity); group_steps: longest run of steps per batch call;
    work_budget: band nodes per step that the running jobs may add up to (a
    job joins when it fits, or when nothing is running); prefetch: jobs that
    may be loading or loaded ahead of joining;
    precision: "fp32" | "fp64" (one per server: a batch has one precision);
    graphs: replay recorded HIP graphs for repeated groups of batch steps;
    batch_streams: streams the batch runs its cache groups on (1 or 2);
    policy: "arrival" (loaded jobs join in arrival order while the work
    budget allows) or "shortest" (at every boundary the jobs with the least
    remaining work run, up to short_budget band nodes per step, or up to
    work_budget while at least busy_backlog requests wait; a running job
    with more left is parked, kept on the device, until the shorter ones
    are done; a job that has waited max_wait_s joins and stays until it is
    done)."""

    def __init__(self, budget_bytes=None, max_active=64, group_steps=10, precision="fp32",
                 load_streams=2, max_reinit_iters=32, work_budget=8_000_000, prefetch=3,
                 graphs=True, batch_streams=2, policy="shortest", short_budget=1_000_000,
                 max_wait_s=0.5, busy_backlog=8):
        if policy not in ("arrival", "shortest"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        self.short_budget = short_budget
        self.max_wait_s = max_wait_s
        self.busy_backlog = busy_backlog
        import torch
        self.torch = torch
        self.precision = precision
        self.graphs = graphs
        self.batch_streams = batch_streams
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget_bytes = budget_bytes
        self.max_active = max_active
        self.group_steps = group_steps
        self.max_reinit_iters = max_reinit_iters
        self.work_budget = work_budget
        self.prefetch = prefetch
        self.batch_stream = torch.cuda.Stream()
        self.load_streams = [torch.cuda.Stream() for _ in range(load_streams)]
        self._next_load = 0

    def _start(self, live):
        """Take the workspace and enqueue the cloud, d and phi0 on a side stream."""
        torch = self.torch
        req = live.req
        s = self.load_streams[self._next_load % len(self.load_streams)]
        self._next_load += 1
        with torch.cuda.stream(s):
            job = lsr.Job(req["grid"], job_params(req, self.precision),
                          max_points=len(req["points"]), stream=s)
            pts = torch.from_numpy(np.ascontiguousarray(req["points"], dtype=np.float64))
            live.pts = pts.pin_memory().to(device=s.device, non_blocking=True)
            lsr.lsr_load_cloud(job.handle, live.pts.data_ptr(), live.pts.shape[0])
            kind = {"sphere": lsr.LSR_PHI_SPHERE, "torus": lsr.LSR_PHI_TORUS}[req["phi0"][0]]
            lsr.lsr_init_phi(job.handle, None, kind, list(req["phi0"][1]), 0)
            live.ev = torch.cuda.Event()
            live.ev.record(s)
        live.job = job
        live.left = int(req["steps"])
        live.state = "loading"

    def _finish(self, live):
        """Copy phi and the band out on the job's own stream."""
        torch = self.torch
        job = live.job
        with torch.cuda.stream(job.stream):
            live.phi = torch.empty(job.nodes, dtype=job.dtype, device=job.stream.device)
            live.band = torch.empty(job.nodes, dtype=torch.uint8, device=job.stream.device)
            lsr.lsr_extract(job.handle, live.phi.data_ptr(), live.band.data_ptr(),
                            want_count=False)
            live.ev = torch.cuda.Event()
            live.ev.record(job.stream)
        live.state = "finishing"

    def run(self, requests, time_scale=1.0, keep_results=False, on_done=None):
        """Serve the requests (each with an "arrival" time in seconds, scaled by
        time_scale) in real time.  Returns a summary dict; with keep_results,
        summary["results"][i] = (phi, band) on the host for request i."""
        torch = self.torch
        order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival"])
        adm = Admission(self.budget_bytes, self.max_active)
        batch = lsr.Batch(max_jobs=self.max_active, group_steps=self.group_steps,
                          max_reinit_iters=self.max_reinit_iters, stream=self.batch_stream)
        batch.set_graphs(self.graphs)
        batch.set_streams(self.batch_streams)
        lives = {}
        pending = collections.deque(order)
        running = []
        finishing = []
        loading = []
        ready = collections.deque()
        work = {}
        running_work = 0
        latency = {}
        results = {}
        done_at = {}
        started_at = {}
        in_flight = collections.deque()  # events of issued batch calls
        waiting_since = {}  # loaded jobs not in the batch: since when
        sticky = set()      # jobs that waited too long: they run until done
        parked = set()      # jobs that ran and were set aside for shorter ones
        keep_set = set()
        n_parked = 0
        n_done = 0
        max_running = 0
        t0 = time.perf_counter()
        first_arrival = None

        def now():
            return time.perf_counter() - t0

        while n_done + len(adm.rejected) < len(requests):
            t = now()
            # arrivals
            while pending and requests[pending[0]]["arrival"] * time_scale <= t:
                i = pending.popleft()
                if first_arrival is None:
                    first_arrival = requests[i]["arrival"] * time_scale
                adm.offer(i, footprint_bytes(requests[i], self.precision))
                work[i] = band_estimate(requests[i])
            # admission: start loading on a side stream
            for i in adm.admit(limit=max(0, self.prefetch - len(loading) - len(ready) + len(parked))):
                live = _Live()
                live.req = requests[i]
                lives[i] = live
                started_at[i] = now()
                self._start(live)
                loading.append(i)
            # loaded jobs become ready; ready jobs join the batch in arrival
            # order while the step's work fits
            for i in [i for i in loading if lives[i].ev.query()]:
                loading.remove(i)
                lives[i].state = "ready"
                ready.append(i)
                waiting_since[i] = now()
            if self.policy == "shortest" and ready:
                # the jobs with the least work left run, up to the short
                # budget; a job that has waited max_wait_s joins them and
                # stays until it is done
                t_now = now()
                for i in ready:
                    if t_now - waiting_since[i] > self.max_wait_s:
                        sticky.add(i)
                backlog = len(adm.queue) + len(loading) + len(ready)  # arrived, waiting
                budget = self.work_budget if backlog >= self.busy_backlog else self.short_budget
                cands = running + list(ready)
                keep = least_work_first(cands, {i: lives[i].left * work[i] for i in cands}, work,
                                        sticky, budget)
                for i in [i for i in running if i not in keep]:
                    batch.remove(lives[i].job)  # parked: its state stays on the device
                    running.remove(i)
                    running_work -= work[i]
                    lives[i].state = "ready"
                    ready.append(i)
                    waiting_since[i] = t_now
                    parked.add(i)
                    n_parked += 1
                ready = collections.deque([i for i in keep if i not in running] +
                                          [i for i in ready if i not in keep])
                keep_set = set(keep)
            while ready:
                i = ready[0]
                w = work[i]
                if self.policy == "shortest":
                    # the order above decided; stop at the first one left out
                    if i not in keep_set:
                        break
                elif running and running_work + w > self.work_budget:
                    break
                ready.popleft()
                waiting_since.pop(i, None)
                parked.discard(i)
                live = lives[i]
                batch.add(live.job, live.req["dt"], live.req["interp"])
                live.state = "running"
                running.append(i)
                running_work += w
            # finished copies: record completion, free the budget
            for i in [i for i in finishing if lives[i].ev.query()]:
                finishing.remove(i)
                live = lives[i]
                done_at[i] = now()
                latency[i] = done_at[i] - live.req["arrival"] * time_scale
                if keep_results:
                    results[i] = (live.phi.cpu().numpy(), live.band.cpu().numpy())
                if on_done is not None:
                    on_done(i, live)
                live.job.close()
                live.job = live.phi = live.band = live.pts = live.ev = None
                adm.release(i)
                n_done += 1
            if running:
                max_running = max(max_running, len(running))
                # keep at most two batch calls in flight
                while len(in_flight) >= 2:
                    in_flight.popleft().synchronize()
                n = min(self.group_steps, min(lives[i].left for i in running))
                batch.step(n)
                ev = torch.cuda.Event()
                ev.record(self.batch_stream)
                in_flight.append(ev)
                for i in list(running):
                    lives[i].left -= n
                    if lives[i].left == 0:
                        batch.remove(lives[i].job)
                        running.remove(i)
                        running_work -= work[i]
                        self._finish(lives[i])
                        finishing.append(i)
            elif loading or finishing:
                # nothing to step: wait for the oldest outstanding event
                lives[(loading or finishing)[0]].ev.synchronize()
            elif pending:
                dt = requests[pending[0]]["arrival"] * time_scale - now()
                if dt > 0:
                    time.sleep(min(dt, 0.01))
        batch.close()
        torch.cuda.synchronize()
        wall = (max(done_at.values()) - first_arrival) if done_at else 0.0
        lat = [1e3 * latency[i] for i in sorted(latency)]
        out = {"jobs": n_done, "rejected": list(adm.rejected), "wall_s": wall,
               "jobs_per_s": n_done / wall if wall > 0 else None,
               "latency_ms": _percentiles(lat), "max_batch": max_running, "parked": n_parked,
               "latency_ms_each": {i: 1e3 * latency[i] for i in latency}}
        if keep_results:
            out["results"] = results
        return out


def run_sequential(requests, precision="fp32", time_scale=1.0, keep_results=False, graphs=True):
    """The same stream served one plain solve at a time (no batching, no
    overlap): the reference the served form is compared with."""
    import torch
    order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival"])
    t0 = time.perf_counter()
    latency, results, done_at = {}, {}, {}
    first = None
    s = torch.cuda.Stream()  # not the null stream: step loops run as graphs
    for i in order:
        req = requests[i]
        arr = req["arrival"] * time_scale
        first = arr if first is None else first
        wait = arr - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        with torch.cuda.stream(s):
            job = lsr.Job(req["grid"], job_params(req, precision),
                          max_points=len(req["points"]), stream=s)
            job.set_graphs(graphs)
            pts = torch.as_tensor(np.ascontiguousarray(req["points"], dtype=np.float64),
                                  device=s.device)
            lsr.lsr_load_cloud(job.handle, pts.data_ptr(), pts.shape[0])
            kind = {"sphere": lsr.LSR_PHI_SPHERE, "torus": lsr.LSR_PHI_TORUS}[req["phi0"][0]]
            lsr.lsr_init_phi(job.handle, None, kind, list(req["phi0"][1]), 0)
            lsr.lsr_step(job.handle, int(req["steps"]), req["dt"],
                         lsr.interp_code(req["interp"]))
            phi = torch.empty(job.nodes, dtype=job.dtype, device=s.device)
            band = torch.empty(job.nodes, dtype=torch.uint8, device=s.device)
            lsr.lsr_extract(job.handle, phi.data_ptr(), band.data_ptr(), want_count=False)
        s.synchronize()
        done_at[i] = time.perf_counter() - t0
        latency[i] = done_at[i] - arr
        if keep_results:
            results[i] = (phi.cpu().numpy(), band.cpu().numpy())
        job.close()
    wall = max(done_at.values()) - first
    lat = [1e3 * latency[i] for i in sorted(latency)]
    out = {"jobs": len(order), "wall_s": wall, "jobs_per_s": len(order) / wall,
           "latency_ms": _percentiles(lat), "latency_ms_each": {i: 1e3 * latency[i] for i in latency}}
    if keep_results:
        out["results"] = results
    return out


def materialise(specs):
    """Requests from synth.served_jobs descriptions: draws each cloud."""
    from . import synth
    out = []
    for r in specs:
        q = dict(r)
        if "points" not in q:
            q["points"] = synth.make_cloud(q["cloud"])
        out.append(q)
    return out
