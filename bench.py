#!/usr/bin/env python3
"""Benchmark of the narrow-band semi-Lagrangian level-set solver on one MI355X.

One bench step = one whole reconstruction of the 3D non-uniform workload
(256^3 grid on [-1,1]^3, 200k points on the union of a sphere and an
ellipsoid with a 10x density ramp and two holes, WENO, dt = h/2, 400 steps,
band 6h, reinitialisation every 10 steps, FP32 state): exact distance field
from the cloud, initial data and first band, 400 time steps (update, band
rebuild, reinitialisation and cut) and the copy-out of phi and the band.  The
cloud is resident in HBM before the timed region.

value = node updates (sum of band sizes over the steps) per second of wall
time over the timed jobs.  The roofline object describes the dominant kernel
(the 3D WENO step), timed with HIP events tied to each launch's dispatch.
The cpu_baseline object times the FP64 oracle's step loop on a bounded
sample of the same workload on the host's cores (all of them and one).
Context objects: the 128^3 torus and the 2D circle workloads, the same jobs
at p = 2, "batched" (many independent jobs in one batch against the same
jobs run one after the other) and "served" (a request stream with continuous
batching against the same stream served by plain solves: every request
queued at once for jobs/s, and a Poisson stream at 20/s for latency).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of one node update of the step kernel (FMA = 2 flops):
# 3D WENO: 84 one-dimensional WENO evaluations x 30 flops, 4 foot points x 42
# flops of per-foot set-up, 60 flops of per-node set-up.
FLOPS_PER_UPDATE = {(3, "weno"): 84 * 30 + 4 * 42 + 60, (3, "q1"): 4 * (7 * 3 + 18) + 60,
                    (2, "weno"): 2 * (5 * 30 + 28) + 40, (2, "q1"): 2 * (3 * 3 + 12) + 40}
# Compulsory HBM bytes of one node update: list entry in 4, phi^n_j e,
# (grad d, d) 4e, phi^{n+1}_j e, list entry out 4, with e the element size.
BYTES_PER_UPDATE = {"fp32": 4 + 4 + 16 + 4 + 4, "fp64": 4 + 8 + 32 + 8 + 4}
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}  # MI355X published vector peaks
PEAK_HBM_GBS = 8000.0
N_CU, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock
DEFAULT_LANES = {2: 1, 3: 1}  # the library's default launch shape (lsr_create)
KERNEL_SOURCES = ["paper_2410_22205_amd/csrc/lsr_device.h", "paper_2410_22205_amd/csrc/lsr_kern.h",
                  "paper_2410_22205_amd/csrc/lsr_step.hip", "paper_2410_22205_amd/csrc/lsr_internal.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_path(workload, precision):
    return os.path.join(ROOT, "profiles", f"sl_step_weno3_{workload}_{precision}_traffic.txt")


def read_profile(workload, precision):
    """The step kernel's committed rocprofv3 counter summary as key: value
    pairs, if it was taken on the current kernel sources, else {}."""
    path = traffic_path(workload, precision)
    if not os.path.exists(path):
        return {}
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv if kv.get("kernel_source_hash") == kernel_source_hash() else {}


def profile_value(kv, key):
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def read_traffic(workload, precision):
    """HBM bytes per launch of the step kernel (FETCH_SIZE and WRITE_SIZE with
    the copy calibration) from the committed summary, or None."""
    return profile_value(read_profile(workload, precision), "hbm_bytes_per_launch")


def run_p2(w, precision, n_jobs, pts):
    """Whole jobs of the workload at p = 2 (one warm-up, n_jobs timed)."""
    import torch

    from paper_2410_22205_amd import lsr
    prm = dict(gamma=w["gamma"], beta=w["beta"], reinit_every=w["reinit_every"], p=2.0,
               precision=precision)
    job = lsr.Job(w["grid"], prm, max_points=len(w["points"]), stream=torch.cuda.Stream())
    kind = {"sphere": lsr.LSR_PHI_SPHERE, "torus": lsr.LSR_PHI_TORUS}[w["phi0"][0]]
    interp = lsr.interp_code(w["interp"])
    torch.cuda.synchronize()

    def one():
        lsr.lsr_load_cloud(job.handle, pts.data_ptr(), pts.shape[0])
        lsr.lsr_init_phi(job.handle, None, kind, list(w["phi0"][1]), 0)
        lsr.lsr_step(job.handle, w["steps"], w["dt"], interp)

    one()
    job.stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_jobs):
        one()
    job.stream.synchronize()
    wall = time.perf_counter() - t0
    # the counters restart with every job, and the jobs are identical
    upd = n_jobs * lsr.lsr_counters(job.handle)["node_updates"]
    e2 = job.energy(2.0)
    job.close()
    return {"jobs": n_jobs, "ms_per_job": 1e3 * wall / n_jobs, "node_updates_per_s": upd / wall,
            "E_2_final": e2}


def host_cpu():
    """Model name and online CPU count of the host (lscpu's fields)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, steps_all=10, steps_one=2):
    """The oracle's step loop (Algorithm 1, step 4: band, update, the
    reinitialisation every K steps and the cut; no distance field and no
    phi0 in the timed region) on the same workload, from phi0: steps_all
    steps on all host cores, steps_one steps on one thread.  The oracle's
    distance field is computed, untimed, only at the nodes those steps can
    read: within the band of phi0 moved by the steps, plus the reach of the
    foot points and of the stencils; the others hold +inf, and a finite
    result shows that no step read one."""
    import numpy as np

    import oracle
    g = w["grid"]
    h = g["h"]
    prm = oracle.default_params(g["dim"], h, gamma=w["gamma"], beta=w["beta"],
                                reinit_every=w["reinit_every"])
    kind, args = w["phi0"]
    phi0 = oracle.init_phi(g, kind, args, prm["gamma"])
    X = oracle.node_coords(g)
    c = np.asarray(args[:g["dim"]])
    if kind == "sphere":
        sdf = np.linalg.norm(X - c, axis=1) - args[3]
    else:
        rho = np.linalg.norm((X - c)[:, :2], axis=1) - args[3]
        sdf = np.sqrt(rho * rho + (X - c)[:, 2] ** 2) - args[4]
    reach = prm["gamma"] + max(steps_all, steps_one) * w["dt"] + 16 * h
    near = np.abs(sdf) < reach
    d = np.full(X.shape[0], np.inf)
    d[near] = oracle.distance(w["points"], g, x=X[near])
    d = d.reshape(phi0.shape)
    out = {}
    for label, threads, k in (("all_cores", 0, steps_all), ("one_thread", 1, steps_one)):
        used = oracle.threads(threads) if threads else oracle.threads(len(os.sched_getaffinity(0)))
        t0 = time.perf_counter()
        phi, counts = oracle.run(phi0, d, g, prm, w["dt"], w["interp"], k)
        dt = time.perf_counter() - t0
        assert np.isfinite(phi).all(), "a sampled step read the distance outside the sample"
        out[label] = {"value": int(counts[0]) / dt, "threads": used, "steps": k,
                      "node_updates": int(counts[0]), "seconds": round(dt, 3)}
    oracle.threads(len(os.sched_getaffinity(0)))
    model, ncpu = host_cpu()
    a = out["all_cores"]
    return {"value": a["value"], "unit": "node-updates/s", "cores": a["threads"], "kind": "oracle",
            "one_thread": out["one_thread"], "host": {"model": model, "nproc": ncpu},
            "sample": (f"the oracle's step loop (FP64, C with OpenMP over band nodes) from phi0 of "
                       f"the same workload: {a['steps']} steps ({a['node_updates']} node updates, "
                       f"one reinitialisation) in {a['seconds']} s on {a['threads']} threads, "
                       f"and {out['one_thread']['steps']} steps on one thread; distance field "
                       f"and phi0 untimed")}


def run_batched(n_jobs, steps, precision, graphs=True, batch_streams=2, phases=("seq", "batch")):
    """The batched workload: independent jobs with uneven grids (64^3-192^3),
    clouds of 5k-150k points, Q1 and WENO alternating, `steps` steps each;
    one after the other as plain solves, then all in one batch (loads on
    side streams, autotuned launch shape).  Wall time from the first cloud
    load to the last extract; the clouds are resident in HBM before either
    timed region."""
    import numpy as np
    import torch
    from paper_2410_22205_amd import lsr, synth
    jobs = synth.batch_jobs(n_jobs=n_jobs, steps=steps)
    pts = [torch.as_tensor(w["points"], dtype=torch.float64, device="cuda").contiguous()
           for w in jobs]
    kinds = {"sphere": lsr.LSR_PHI_SPHERE, "torus": lsr.LSR_PHI_TORUS}

    seq_stream = torch.cuda.Stream()  # streams of their own: step loops run as graphs

    def make(w):
        job = lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"],
                                      reinit_every=w["reinit_every"], precision=precision),
                      max_points=len(w["points"]), stream=seq_stream)
        job.set_graphs(graphs)
        return job

    def load(job, w, p):
        lsr.lsr_load_cloud(job.handle, p.data_ptr(), p.shape[0])
        lsr.lsr_init_phi(job.handle, None, kinds[w["phi0"][0]], list(w["phi0"][1]), 0)

    def extract(job):
        phi = torch.empty(job.nodes, dtype=job.dtype, device="cuda")
        band = torch.empty(job.nodes, dtype=torch.uint8, device="cuda")
        lsr.lsr_extract(job.handle, phi.data_ptr(), band.data_ptr(), want_count=False)
        return phi, band

    # one after the other
    upd = 0
    t_seq = float("nan")
    if "seq" in phases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(seq_stream):
            for w, p in zip(jobs, pts):
                job = make(w)
                load(job, w, p)
                lsr.lsr_step(job.handle, w["steps"], w["dt"], lsr.interp_code(w["interp"]))
                extract(job)
                upd += lsr.lsr_counters(job.handle)["node_updates"]
                job.close()
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
    if "batch" not in phases:
        return {"sequential_jobs_per_s": n_jobs / t_seq}
    # all in one batch; the jobs load (distance field, phi0) on four side
    # streams so that the loads of small jobs overlap
    streams = [torch.cuda.Stream() for _ in range(4)]
    handles = []
    for k, w in enumerate(jobs):
        with torch.cuda.stream(streams[k % 4]):
            handles.append(lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"],
                                                   reinit_every=w["reinit_every"],
                                                   precision=precision),
                                   max_points=len(w["points"]), stream=streams[k % 4]))
    # the launch shape is tuned once for this batch signature before the
    # timed region (as a deployment would, or from lsr_set_tune_cache)
    bstream = torch.cuda.Stream()
    for job, w, p in zip(handles, jobs, pts):
        load(job, w, p)
    probe = lsr.Batch(max_jobs=n_jobs, group_steps=10, stream=bstream)
    for job, w in zip(handles, jobs):
        probe.add(job, w["dt"], w["interp"])
    probe.tune()
    probe.close()
    batch = lsr.Batch(max_jobs=n_jobs, group_steps=10, stream=bstream)
    batch.set_graphs(graphs)
    batch.set_streams(batch_streams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for job, w, p in zip(handles, jobs, pts):
        load(job, w, p)
    for job, w in zip(handles, jobs):
        batch.add(job, w["dt"], w["interp"])
    lanes, bpc, _ = batch.tune()
    batch.step(steps)
    graphs = batch.graph_counts()
    for job in list(handles):
        batch.remove(job)
        extract(job)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    upd_b = sum(lsr.lsr_counters(j.handle)["node_updates"] for j in handles)
    assert "seq" not in phases or upd_b == upd, "batched and sequential runs did different work"
    upd = upd_b
    batch.close()
    for j in handles:
        j.close()
    return {"workload": f"{n_jobs} jobs, grids 64^3-192^3, 5k-150k points, Q1/WENO alternating, "
                        f"{steps} steps each, dt = h/2, reinit every 10",
            "jobs_per_s": n_jobs / t_bat, "sequential_jobs_per_s": n_jobs / t_seq,
            "speedup": t_seq / t_bat, "node_updates_per_s": upd / t_bat,
            "sequential_node_updates_per_s": upd / t_seq,
            "tuned": {"lanes": lanes, "blocks_per_cu": bpc},
            "group_graphs": dict(zip(("recorded", "replays"), graphs))}


def run_served(n_jobs, precision, graphs=True, streams=2):
    """The served workload: a stream of jobs with grids 64^3-320^3, 5k-1M
    points, 200-400 WENO steps, served with continuous batching (the
    server's default policy: least work left first) and as plain solves one
    at a time, each way twice: with every request queued at once (the
    capacity in jobs/s), and arriving as a Poisson stream at 20 requests/s
    (latency = completion - arrival, p50/p99)."""
    from paper_2410_22205_amd import serve, synth
    reqs = serve.materialise(synth.served_jobs(n_jobs=n_jobs))
    srv = serve.Server(precision=precision, graphs=graphs, batch_streams=streams)
    warm = serve.materialise(synth.served_jobs(n_jobs=2, seed=77))
    srv.run([dict(r, arrival=0.0) for r in warm])
    at_once = [dict(r, arrival=0.0) for r in reqs]
    cap = srv.run(at_once)
    cap_seq = serve.run_sequential(at_once, precision=precision, graphs=graphs)
    out = srv.run(reqs)
    seq = serve.run_sequential(reqs, precision=precision, graphs=graphs)
    return {"workload": f"{n_jobs} requests, grids 64^3-320^3, 5k-1M points, WENO, 200-400 steps",
            "jobs_per_s": cap["jobs_per_s"], "sequential_jobs_per_s": cap_seq["jobs_per_s"],
            "speedup": cap["jobs_per_s"] / cap_seq["jobs_per_s"],
            "max_batch": cap["max_batch"], "rejected": len(cap["rejected"]),
            "poisson_20_per_s": {
                "jobs_per_s": out["jobs_per_s"], "latency_ms": out["latency_ms"],
                "max_batch": out["max_batch"], "rejected": len(out["rejected"]),
                "sequential": {"jobs_per_s": seq["jobs_per_s"], "latency_ms": seq["latency_ms"]}}}


def workload_config(name, w):
    g = w["grid"]
    return {"workload": name, "grid": "x".join(str(v) for v in g["n"]),
            "points": len(w["points"]), "interp": w["interp"],
            "dt": "h/2" if g["dim"] == 3 else "h", "steps_per_job": w["steps"], "band": "6h",
            "reinit_every": w["reinit_every"], "parallelism": "single GPU"}


def measure(name, precision, n_jobs, warmup, lanes=-1, blocks_per_cu=8, graphs=True):
    """Whole jobs of one workload (distance field, phi0 and first band, all
    steps, copy-out of phi and the band mask), the cloud resident in HBM:
    `warmup` jobs through the step-loop graphs, then `n_jobs` timed jobs with
    every step kernel timed by events tied to its dispatch.  Returns the
    workload, the (open) job and the timings."""
    import torch

    from paper_2410_22205_amd import lsr, synth
    w = synth.workload(name)
    g = w["grid"]
    dim = g["dim"]
    prm = dict(gamma=w["gamma"], beta=w["beta"], reinit_every=w["reinit_every"],
               precision=precision)
    # a stream of its own (the null stream cannot be captured into graphs)
    job = lsr.Job(g, prm, max_points=len(w["points"]), stream=torch.cuda.Stream())
    if lanes > 0 or blocks_per_cu != 8:
        lsr.lsr_set_launch(job.handle, lanes if lanes > 0 else DEFAULT_LANES[dim], blocks_per_cu)
    lanes = lanes if lanes > 0 else DEFAULT_LANES[dim]
    if not graphs:
        job.set_graphs(False)
    stream = job.stream
    pts = torch.as_tensor(w["points"], dtype=torch.float64, device="cuda").contiguous()
    phi_out = torch.empty(job.nodes, dtype=job.dtype, device="cuda")
    band_out = torch.empty(job.nodes, dtype=torch.uint8, device="cuda")
    kind = {"sphere": lsr.LSR_PHI_SPHERE, "torus": lsr.LSR_PHI_TORUS}[w["phi0"][0]]
    interp = lsr.interp_code(w["interp"])
    torch.cuda.synchronize()  # inputs uploaded on torch's stream before the job's stream reads them

    def one_job():
        lsr.lsr_load_cloud(job.handle, pts.data_ptr(), pts.shape[0])
        lsr.lsr_init_phi(job.handle, None, kind, list(w["phi0"][1]), 0)
        lsr.lsr_step(job.handle, w["steps"], w["dt"], interp)
        lsr.lsr_extract(job.handle, phi_out.data_ptr(), band_out.data_ptr(), want_count=False)

    for _ in range(warmup):
        one_job()
    stream.synchronize()
    warm_updates = lsr.lsr_counters(job.handle)["node_updates"] if warmup else None
    lsr.lsr_profile_enable(job.handle, True, w["steps"] * n_jobs + 8)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_jobs):
        ts = time.perf_counter()
        one_job()
        stream.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms, launches = lsr.lsr_profile_read(job.handle)
    lsr.lsr_profile_enable(job.handle, False)
    # the counters restart with every initialisation: they hold the last job's
    updates = lsr.lsr_counters(job.handle)["node_updates"]
    assert warm_updates is None or warm_updates == updates, "runs are not deterministic"
    job.pts = pts
    return w, job, {"wall": wall, "kernel_ms": kernel_ms, "launches": launches, "lat": lat,
                    "updates_per_job": updates, "lanes": lanes}


def context_line(name, precision, n_jobs):
    """A smaller workload as context: whole jobs and the step kernel's rate."""
    w, job, r = measure(name, precision, n_jobs, 1)
    job.close()
    upd = r["updates_per_job"] * n_jobs
    lat_ms = sorted(1e3 * x for x in r["lat"])
    return {"config": workload_config(name, w), "jobs": n_jobs,
            "ms_per_job": 1e3 * r["wall"] / n_jobs, "node_updates_per_s": upd / r["wall"],
            "sl_kernel_node_updates_per_s": upd / (r["kernel_ms"] / 1e3),
            "sl_kernel_avg_launch_us": round(r["kernel_ms"] * 1e3 / r["launches"], 3),
            "node_updates_per_job": r["updates_per_job"],
            "latency_ms": {"p50": lat_ms[len(lat_ms) // 2], "max": lat_ms[-1]}}


def copy_calibration():
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings (run under rocprofv3 --pmc)."""
    import torch
    n = 256 << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n, "copy_bytes_written_per_launch": n,
                      "launches": 5}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed jobs")
    ap.add_argument("--p2-jobs", type=int, default=2,
                    help="timed jobs of the same workload at p = 2 (context; 0 = skip)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="union3d")
    ap.add_argument("--context-jobs", type=int, default=3,
                    help="timed jobs of the other single-job workloads (context; 0 = skip)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--lanes", type=int, default=-1,
                    help="step kernel: 1 one lane per node, 4 (2 in 2D) one lane per foot point; "
                         "-1 the library default")
    ap.add_argument("--blocks-per-cu", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel directly")
    ap.add_argument("--batch-streams", type=int, default=2, choices=[1, 2],
                    help="streams a batch runs its cache groups on")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batch-jobs", type=int, default=64, help="batched section (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-phases", default="seq,batch",
                    help="which halves of the batched section run (profiling: seq or batch)")
    ap.add_argument("--served-jobs", type=int, default=400, help="served section (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    w, job, r = measure(args.workload, args.precision, args.steps, args.warmup, args.lanes,
                        args.blocks_per_cu, not args.no_graphs)
    g = w["grid"]
    dim = g["dim"]
    lanes = r["lanes"]
    wall, kernel_ms, launches = r["wall"], r["kernel_ms"], r["launches"]
    updates_per_job = r["updates_per_job"]
    total_updates = updates_per_job * args.steps
    value = total_updates / wall
    kernel_s = kernel_ms / 1e3
    flops = FLOPS_PER_UPDATE[(dim, w["interp"])]
    achieved_tflops = flops * total_updates / kernel_s / 1e12
    upd_per_launch = total_updates / launches
    traffic = read_traffic(args.workload, args.precision)
    peak = PEAK_TFLOPS[args.precision]
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / peak, 4),
                "traffic": traffic,
                "kernel": f"k_sl_step<{dim},{w['interp']},{'double' if args.precision == 'fp64' else 'float'}>",
                "flops_per_node_update": flops,
                "avg_launch_us": round(kernel_ms * 1e3 / launches, 3),
                "node_updates_per_launch": round(upd_per_launch, 1),
                "lanes": lanes, "blocks_per_cu": args.blocks_per_cu}
    # the vector L1's tag lookups (one 128-byte line per cycle per CU) that
    # the step kernel's gathers take, against the launch time measured here
    tags = profile_value(read_profile(args.workload, args.precision),
                         "l1_tag_lookups_per_launch")
    launch_cycles = kernel_ms * 1e-3 / launches * CLOCK_HZ
    l1 = None if tags is None else {
        "tag_lookups_per_launch": tags, "per_cu_cycle": round(tags / N_CU / launch_cycles, 4),
        "peak": 1.0, "unit": "tag lookups per CU per cycle",
        "source": "TCP_TOTAL_CACHE_ACCESSES_sum of the committed counter summary; launch time live"}
    hbm_gbs = BYTES_PER_UPDATE[args.precision] * total_updates / kernel_s / 1e9
    lat_ms = sorted(1e3 * x for x in r["lat"])
    out = {
        "metric": "narrow-band node-updates/s (3D WENO SL step) + jobs/s, p50/p99 latency",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": workload_config(args.workload, w),
        "roofline": roofline,
        "l1": l1,
        "hbm": {"algorithmic_bytes_per_update": BYTES_PER_UPDATE[args.precision],
                "achieved_gbs": round(hbm_gbs, 1),
                "peak_gbs": PEAK_HBM_GBS, "frac": round(hbm_gbs / PEAK_HBM_GBS, 4)},
        "sl_kernel_node_updates_per_s": total_updates / kernel_s,
        "sl_kernel_share_of_wall": kernel_s / wall,
        "node_updates_per_job": updates_per_job,
        "jobs_per_s": args.steps / wall,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
    }
    # E_2 of the last job's final phi (Section 3.5), outside the timed
    # region: this workload runs at p = 1 for a fixed step count, so its loop
    # needs no energy.  Wall time per call includes the 8-byte copy back and
    # the synchronisation; the kernels' own time is in the rocprofv3 trace.
    e2 = job.energy(2.0)
    t0 = time.perf_counter()
    for _ in range(10):
        job.energy(2.0)
    out["energy"] = {"p": 2, "R": 5, "E_p": e2,
                     "wall_us_per_call": round((time.perf_counter() - t0) / 10 * 1e6, 1)}
    # the cloud resolution h_S over a seeded 10 % sample (Section 4), also
    # outside the timed region: preprocessing, not part of the loop
    sample = np.random.default_rng(11).choice(len(w["points"]), size=len(w["points"]) // 10,
                                               replace=False)
    h_s = job.cloud_spacing(sample)
    t0 = time.perf_counter()
    for _ in range(10):
        job.cloud_spacing(sample)
    out["cloud_spacing"] = {"h_S": h_s, "sample": int(len(sample)),
                            "wall_us_per_call": round((time.perf_counter() - t0) / 10 * 1e6, 1)}
    job_pts = job.pts
    job.close()
    job.pts = job_pts
    # context, not the headline: the same jobs at p = 2, where every step
    # first computes E_2 of the current phi on the device
    if args.p2_jobs:
        out["p2"] = run_p2(w, args.precision, args.p2_jobs, job.pts)
    # the other single-job workloads, as context
    if args.context_jobs:
        out["context"] = {name: context_line(name, args.precision, args.context_jobs)
                          for name in ("torus3d", "circle2d") if name != args.workload}
    if args.batch_jobs:
        out["batched"] = run_batched(args.batch_jobs, args.batch_steps, args.precision,
                                     graphs=not args.no_graphs,
                                     batch_streams=args.batch_streams,
                                     phases=tuple(args.batch_phases.split(",")))
    if args.served_jobs:
        out["served"] = run_served(args.served_jobs, args.precision, graphs=not args.no_graphs,
                                   streams=args.batch_streams)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
