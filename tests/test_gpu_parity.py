"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, for both state precisions of the library.

Tolerances: the distance field within 4 double ulps of the exact value (the
minimum is exact, the distance arithmetic is summed in another order);
one step within 1e-5 h; whole runs within 1e-4 h (max |phi_gpu - phi_oracle|);
band membership bit-exact except for nodes whose oracle value lies within
1e-6 h of the band threshold gamma.

On the 128^3 torus and the 256^3 union workloads the scheme itself is
unstable to rounding: on the torus the front reaches the torus axis, where d
has a cone point; on the union the e2-based tangent frame of eq. (sigma3d) is
ill-conditioned near the poles of the initial sphere (sqrt(d1 phi^2 +
d3 phi^2) small, so a rounding change turns the frame).  The FP64 oracle
started from phi0 perturbed by one ulp differs from itself by O(h) after ~35
steps on the torus and by 0.4 h after 20 on the union (pinned, at 128^3
and at 96^3, by tests/test_oracle_sensitivity.py).  No implementation that does not repeat
the oracle's exact operation order can stay within 1e-4 h over such runs.
They are therefore held to:
  * 1e-4 h from phi0 over the horizon before the divergence;
  * stepwise parity over the whole run: after every step the device's state
    equals the oracle's single step (band, update, reinitialisation and cut)
    taken from the device's previous state, within 1e-10 h in FP64 (about
    1e5 ulps of gamma; every discrete disagreement seen so far, a band or
    interface decision or a frame branch, moves a node by 1e-3 h or more);
  * the same attachment to the cloud at the end of the run.
Workloads without the instability (the 2D circle, the torus at 48^3) are
held to 1e-4 h over the whole run.
"""
import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu


def _lsr():
    from paper_2410_22205_amd import lsr
    return lsr


PRECISIONS = ["fp32", "fp64"]


def gpu_run(w, steps=None, d=None, step0=0, extra=None, precision="fp64"):
    lsr = _lsr()
    oprm = oracle_params(w, extra)
    prm = {k: oprm[k] for k in ("p", "gamma", "beta", "reinit_every", "reinit_iters",
                                "reinit_dtau", "delta", "grad_C", "grad_alpha", "interface_floor")}
    prm["precision"] = precision
    job = lsr.Job(w["grid"], prm, max_points=len(w["points"]))
    if d is None:
        job.load_cloud(w["points"])
    else:
        job.set_distance(d)
    if w["phi0"][0] == "array":
        job.init_phi(phi0=w["phi0"][1], step0=step0)
    else:
        job.init_phi(w["phi0"][0], w["phi0"][1], step0=step0)
    n = w["steps"] if steps is None else steps
    if n:
        job.step(n, w["dt"], w["interp"])
    phi, band, nb, si = job.extract()
    cnt = job.counters()
    dgpu = job.distance()
    job.close()
    return phi, band, nb, si, cnt, dgpu


def oracle_params(w, extra=None):
    g = w["grid"]
    prm = oracle.default_params(g["dim"], g["h"], gamma=w["gamma"], beta=w["beta"],
                                reinit_every=w["reinit_every"])
    prm.update(extra or {})
    return prm


def oracle_run(w, steps=None, d=None, extra=None):
    g = w["grid"]
    prm = oracle_params(w, extra)
    if d is None:
        d = oracle.distance(w["points"], g)
    if w["phi0"][0] == "array":
        phi0 = np.clip(np.asarray(w["phi0"][1], np.float64), -prm["gamma"], prm["gamma"])
    else:
        phi0 = oracle.init_phi(g, w["phi0"][0], w["phi0"][1], prm["gamma"])
    n = w["steps"] if steps is None else steps
    phi, counts = oracle.run(phi0, d, g, prm, w["dt"], w["interp"], n)
    return phi, counts, d, prm


def check_phi(phi_gpu, phi_orc, h, tol):
    err = np.abs(phi_gpu.astype(np.float64) - phi_orc)
    worst = float(err.max())
    where = np.unravel_index(int(err.argmax()), err.shape)
    assert worst <= tol * h, f"max |dphi| = {worst / h:.3e} h at {where} (tol {tol:g} h)"
    return worst / h


def check_band(band_gpu, phi_gpu, phi_orc, gamma, h, margin=1e-6):
    """The device's own band list is exactly {|phi_gpu| < gamma} in its
    precision, and agrees with the oracle's band at every node whose oracle
    value lies farther than margin * h from gamma (1e-6 h; for an FP32 state
    compared step by step, the value bar of that comparison, since the
    values themselves differ by up to that)."""
    g = phi_gpu.dtype.type(gamma)
    np.testing.assert_array_equal(band_gpu, (np.abs(phi_gpu) < g).astype(np.uint8))
    want = np.abs(phi_orc) < gamma
    sure = np.abs(np.abs(phi_orc) - gamma) > margin * h
    bad = (band_gpu.astype(bool) != want) & sure
    assert not bad.any(), f"{int(bad.sum())} band nodes differ away from the threshold"


# ------------------------------------------------------------ distance

@pytest.mark.parametrize("name,n", [("circle2d", 128), ("torus3d", 45), ("torus3d", 128)])
def test_distance_field_matches_oracle(name, n):
    w = synth.workload(name, n=n)
    _, _, _, _, _, dgpu = gpu_run(w, steps=0)
    dor = oracle.distance(w["points"], w["grid"])
    err = np.abs(dgpu - dor)
    assert (err <= 4 * np.spacing(dor)).all(), f"max err {err.max():.3e}"


def test_distance_field_union_sampled():
    """256^3, 200k points: sampled nodes against the oracle's exact query."""
    w = synth.workload("union3d")
    _, _, _, _, _, dgpu = gpu_run(w, steps=0)
    g = w["grid"]
    rng = np.random.default_rng(17)
    idx = rng.choice(dgpu.size, size=400_000, replace=False)
    X = np.stack(np.unravel_index(idx, dgpu.shape), 1) * g["h"] + np.array(g["lo"])
    dor = oracle.distance(w["points"], g, x=X)
    got = dgpu.ravel()[idx]
    assert (np.abs(got - dor) <= 4 * np.spacing(dor)).all()


@pytest.mark.parametrize("case", ["dense", "corner", "corner2d", "sphere_centre"])
def test_distance_field_dense_and_far_clouds(case):
    """Many points per bin (80k points on a small torus at 72^3), nodes up to
    the far corner of the grid from a cloud in one corner, and the centre of
    a dense sphere (150k points, about 8000 bins at 128^3), where every bin
    lies at nearly the same distance, so that a brick's candidates overflow
    the kernel's lists: the bins are visited nearest first and skipped wave
    by wave, or walked without order, and every node still gets its exact
    nearest distance."""
    if case == "dense":
        g = synth.cube_grid(3, 72)
        pts = synth.torus_cloud(80_000, 0.3, 0.1, 0.0, seed=21)
    elif case == "sphere_centre":
        g = synth.cube_grid(3, 128)
        pts = synth.sphere_points(np.random.default_rng(24), 150_000, 0.8)
    elif case == "corner":
        g = synth.cube_grid(3, 96)
        pts = synth.torus_cloud(4_000, 0.15, 0.05, 0.0, seed=22) + np.array([-0.75, -0.7, -0.72])
    else:
        g = synth.cube_grid(2, 200)
        pts = synth.circle_cloud(3_000, 0.15, seed=23, centre=(-0.78, -0.74))
    w = dict(grid=g, points=pts, phi0=("sphere", (0.0, 0.0, 0.0, 0.9)), interp="weno",
             dt=0.5 * g["h"], steps=0, gamma=6 * g["h"], beta=3 * g["h"], reinit_every=0)
    _, _, _, _, _, dgpu = gpu_run(w, steps=0)
    if case == "sphere_centre":
        # every node near the centre, where the lists overflow, and a random
        # sample of the rest (the oracle's tree query is slow at the centre)
        X = oracle.node_coords(g)
        near = np.nonzero(np.abs(X).max(axis=1) <= 0.09)[0]
        rest = np.random.default_rng(25).choice(dgpu.size, size=50_000, replace=False)
        idx = np.union1d(near, rest)
        dor = oracle.distance(w["points"], g, x=X[idx])
        got = dgpu.ravel()[idx]
        assert near.size > 1000
        assert (np.abs(got - dor) <= 4 * np.spacing(dor)).all()
        return
    dor = oracle.distance(w["points"], g)
    err = np.abs(dgpu - dor)
    assert (err <= 4 * np.spacing(dor)).all(), f"max err {err.max():.3e}"


# ------------------------------------------------------------ one step

@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,n,interp", [
    ("circle2d", 128, "q1"), ("circle2d", 128, "weno"), ("circle2d", 61, "weno"),
    ("torus3d", 40, "q1"), ("torus3d", 40, "weno"), ("torus3d", 37, "weno"),
])
def test_one_step_matches_oracle(name, n, interp, precision):
    w = synth.workload(name, n=n)
    w["interp"] = interp
    w["reinit_every"] = 0
    h = w["grid"]["h"]
    phi, band, nb, si, cnt, _ = gpu_run(w, steps=1, precision=precision)
    ophi, counts, _, prm = oracle_run(w, steps=1)
    check_phi(phi, ophi, h, 1e-5)
    check_band(band, phi, ophi, prm["gamma"], h)
    assert si == 1 and cnt["node_updates"] == counts[0]


def _ragged_case(centre):
    g = {"dim": 3, "n": (23, 41, 30), "lo": (-0.6, -1.0, -0.75), "h": 0.05}
    pts = synth.torus_cloud(3000, 0.45, 0.18, 0.0, seed=9)
    pts = pts[np.all(np.abs(pts) < [0.5, 0.9, 0.7], axis=1)]
    return dict(grid=g, points=pts, phi0=("sphere", tuple(centre) + (0.5,)), interp="weno",
                dt=0.5 * g["h"], steps=3, gamma=6 * g["h"], beta=3 * g["h"], reinit_every=2)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ragged_anisotropic_grid(precision):
    """Uneven extents (none a multiple of a tile), a box not centred on the
    origin, a reinitialisation inside the run.  The sphere's centre is off
    every grid line, so no node has a gradient along an axis (the frame test
    of eq. (sigma3d) has no ties)."""
    w = _ragged_case((0.0123, 0.0571, -0.0087))
    phi, band, nb, _, cnt, _ = gpu_run(w, precision=precision)
    ophi, counts, _, prm = oracle_run(w)
    check_phi(phi, ophi, w["grid"]["h"], 1e-4)
    check_band(band, phi, ophi, prm["gamma"], w["grid"]["h"])
    assert counts[2] == 0


def test_frame_regularisation_on_a_symmetry_axis():
    """A sphere centred on grid lines: nodes on its axes have a gradient along
    e2 and take the regularised frame (e1, e3).  Whether such a node ties is
    decided by the last bit of phi0 (x = lo + i h is not exact in binary), so
    the branch taken is compared with an FP64 state, where both sides see
    bitwise the same initial data."""
    w = _ragged_case((0.0, 0.05, 0.0))
    phi, band, nb, _, cnt, _ = gpu_run(w, precision="fp64")
    ophi, counts, _, prm = oracle_run(w)
    check_phi(phi, ophi, w["grid"]["h"], 1e-4)
    check_band(band, phi, ophi, prm["gamma"], w["grid"]["h"])
    assert cnt["frame0"] == counts[2] > 0


# ------------------------------------------------------------ whole runs

def _err_cloud(phi, grid, points):
    """Mean |I[phi](Q)| over (every 20th point of) the cloud, eq. (errCloud),
    with Q1 interpolation."""
    return float(np.mean(np.abs(oracle.interp(phi, grid, points[::20], "q1"))))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_run_circle2d(precision):
    """The 2D workload as specified: 128^2, Q1, dt = h, 200 steps, reinit
    after every step."""
    w = synth.workload("circle2d")
    h = w["grid"]["h"]
    phi, band, nb, si, cnt, _ = gpu_run(w, precision=precision)
    ophi, counts, _, prm = oracle_run(w)
    e = check_phi(phi, ophi, h, 1e-4)
    check_band(band, phi, ophi, prm["gamma"], h)
    assert si == 200 and cnt["reinits"] == 200
    print(f"circle2d: max |dphi| = {e:.2e} h, node updates {cnt['node_updates']} vs {counts[0]}")


@pytest.mark.parametrize("interp", ["q1", "weno"])
def test_full_run_torus3d_small(interp):
    w = synth.workload("torus3d", n=48, steps=100)
    w["interp"] = interp
    h = w["grid"]["h"]
    phi, band, nb, si, cnt, _ = gpu_run(w, precision="fp64")
    ophi, counts, _, prm = oracle_run(w)
    check_phi(phi, ophi, h, 1e-4)
    check_band(band, phi, ophi, prm["gamma"], h)
    assert cnt["reinits"] == 10


def _perturbed_oracle(w, d, steps, rel=2.0 ** -52):
    """The oracle from phi0 with every band value moved by a relative rel
    (default one FP64 ulp; 2^-24 for the resolution of an FP32 state)."""
    g = w["grid"]
    prm = oracle_params(w)
    phi0 = oracle.init_phi(g, w["phi0"][0], w["phi0"][1], prm["gamma"])
    rng = np.random.default_rng(1)
    band = np.abs(phi0) < prm["gamma"]
    phi0 = np.where(band, phi0 * (1 + rng.choice([-1.0, 1.0], phi0.shape) * rel), phi0)
    phi, _ = oracle.run(phi0, d, g, prm, w["dt"], w["interp"], steps)
    return phi


def stepwise_errors(w, steps, d, precision="fp64"):
    """Run the device `steps` steps from phi0 with the distance field d,
    reading the state back after every step; return the largest difference
    (in h) between the device's state n+1 and the oracle's one step from the
    device's state n, over the steps, and where it was.  The band is checked
    at every step."""
    lsr = _lsr()
    g = w["grid"]
    h = g["h"]
    oprm = oracle_params(w)
    prm = {k: oprm[k] for k in ("gamma", "beta", "reinit_every", "reinit_iters", "reinit_dtau")}
    prm["precision"] = precision
    if precision == "fp32":
        # an FP32 state holds the plateau at float32(gamma): the oracle stepping
        # from that state decides band membership against the same value
        oprm = dict(oprm, gamma=float(np.float32(oprm["gamma"])))
    job = lsr.Job(g, prm)
    job.set_distance(d)
    job.init_phi(w["phi0"][0], w["phi0"][1])
    prev = job.extract()[0].astype(np.float64)
    worst, where = 0.0, None
    for s in range(steps):
        ref, _ = oracle.run(prev, d, g, oprm, w["dt"], w["interp"], 1, step0=s)
        job.step(1, w["dt"], w["interp"])
        cur, band, nb, si = job.extract()
        err = np.abs(cur.astype(np.float64) - ref)
        assert si == s + 1
        check_band(band, cur, ref, oprm["gamma"], h)
        if err.max() / h > worst:
            worst = float(err.max()) / h
            where = (s + 1, np.unravel_index(int(err.argmax()), err.shape))
        prev = cur.astype(np.float64)
    job.close()
    return worst, where


def test_full_run_torus3d_full_size_fp64():
    """The 3D single-instance workload at full size (128^3, 20k noisy torus
    points, WENO, dt = h/2, reinit every 10 steps), FP64 state: within 1e-4 h
    (and band-exact) from phi0 over the first 25 steps; each of the 300 steps
    within 1e-10 h of the oracle's step from the device's state; after the
    300 steps the mean difference from the oracle's run over the band no
    more than twice what a one-ulp perturbation of phi0 makes it, with the
    same attachment to the cloud."""
    w = synth.workload("torus3d", steps=25)
    h = w["grid"]["h"]
    d = oracle.distance(w["points"], w["grid"])
    phi, band, nb, si, cnt, _ = gpu_run(w, precision="fp64")
    ophi, counts, _, prm = oracle_run(w, d=d)
    e = check_phi(phi, ophi, h, 1e-4)
    check_band(band, phi, ophi, prm["gamma"], h)
    assert cnt["node_updates"] == counts[0]
    w = synth.workload("torus3d")
    step_err, where = stepwise_errors(w, w["steps"], d)
    assert step_err <= 1e-10, (step_err, where)
    phi, band, nb, si, cnt, _ = gpu_run(w, precision="fp64")
    ophi, counts, _, prm = oracle_run(w, d=d)
    pphi = _perturbed_oracle(w, d, w["steps"])
    sel = (np.abs(ophi) < prm["gamma"]) | (np.abs(phi) < prm["gamma"])
    gpu_mean = np.abs(phi - ophi)[sel].mean()
    env_mean = np.abs(pphi - ophi)[sel].mean()
    assert np.abs(pphi - ophi).max() > 1e-4 * h  # the instability is there
    assert gpu_mean <= 2 * env_mean, (gpu_mean / h, env_mean / h)
    eg = _err_cloud(phi, w["grid"], w["points"])
    eo = _err_cloud(ophi, w["grid"], w["points"])
    assert abs(eg - eo) < 0.02 * h
    print(f"torus3d fp64: 25 steps max |dphi| {e:.2e} h; stepwise max {step_err:.2e} h; "
          f"300 steps mean {gpu_mean / h:.2e} h vs oracle envelope mean {env_mean / h:.2e} h; "
          f"Err_S {eg / h:.4f} h vs {eo / h:.4f} h")


def test_fp32_torus3d_full_size():
    """FP32 state on the 128^3 workload: the first steps within 1e-4 h of the
    oracle; each of the 300 steps within 2e-5 h of the oracle's FP64 step
    from the device's FP32 state (band-exact away from the threshold): one
    FP32 update rounds its ~2,700 operations on values up to gamma = 6h, and
    the largest error over the run's 6e7 updates is about 19 FP32 ulps of
    gamma (1.3e-5 h), where the small-grid one-step tests see 1e-5 h; after
    the 300 steps the mean deviation from the oracle over the band is at most
    twice what a 2^-24 relative perturbation of phi0 (the FP32 state's
    resolution) makes the oracle's own run deviate, with the same attachment
    to the cloud (Err_S within 0.02 h) and band work within 1 %."""
    w = synth.workload("torus3d", steps=5)
    h = w["grid"]["h"]
    phi, band, _, _, _, _ = gpu_run(w, precision="fp32")
    d = oracle.distance(w["points"], w["grid"])
    ophi, _, _, prm = oracle_run(w, d=d)
    check_phi(phi, ophi, h, 1e-4)
    step_err, where = stepwise_errors(synth.workload("torus3d"), 300, d, precision="fp32")
    assert step_err <= 2e-5, (step_err, where)
    print(f"fp32 torus3d stepwise max {step_err:.2e} h at {where}")
    w = synth.workload("torus3d")
    phi, band, nb, si, cnt, _ = gpu_run(w, precision="fp32")
    ophi, counts, _, prm = oracle_run(w, d=d)
    pphi = _perturbed_oracle(w, d, w["steps"], rel=2.0 ** -24)
    phi = phi.astype(np.float64)
    sel = (np.abs(ophi) < prm["gamma"]) | (np.abs(phi) < prm["gamma"])
    gpu_mean = np.abs(phi - ophi)[sel].mean()
    env_mean = np.abs(pphi - ophi)[sel].mean()
    assert gpu_mean <= 2 * env_mean, (gpu_mean / h, env_mean / h)
    eg = _err_cloud(phi, w["grid"], w["points"])
    eo = _err_cloud(ophi, w["grid"], w["points"])
    assert abs(eg - eo) < 0.02 * h, (eg / h, eo / h)
    assert abs(cnt["node_updates"] - counts[0]) < 0.01 * counts[0]
    print(f"fp32 torus3d: Err_S gpu {eg / h:.4f} h oracle {eo / h:.4f} h, mean |dphi| "
          f"{gpu_mean / h:.2e} h vs envelope {env_mean / h:.2e} h, max "
          f"{np.abs(phi - ophi).max() / h:.2e} h")


def sampled_stepwise(w, steps, d, precision, n_sample=20000, full_every=5, seed=7):
    """Stepwise parity at full size on sampled nodes, in the launch shape the
    bench times.  After every step the device's values at n_sample nodes of
    the previous band (a fresh seeded sample each step) must equal the
    oracle's update of those nodes from the device's previous state, and a
    sample of the other nodes must have kept their values exactly; the
    device's band mask must be exactly {|phi| < gamma} of its own state.  At
    every full_every-th reinitialisation the whole state is compared with the
    oracle's step plus reinitialisation from the device's previous state,
    band membership included.  Returns (worst sampled error, worst full-check
    error) in units of h and where the worst sampled one was."""
    lsr = _lsr()
    g = w["grid"]
    h = g["h"]
    oprm = oracle_params(w)
    prm = {k: oprm[k] for k in ("gamma", "beta", "reinit_every", "reinit_iters", "reinit_dtau")}
    prm["precision"] = precision
    if precision == "fp32":
        oprm = dict(oprm, gamma=float(np.float32(oprm["gamma"])))
    gam = oprm["gamma"]
    band_margin = 1e-6 if precision == "fp64" else 2e-5
    job = lsr.Job(g, prm)
    job.set_distance(d)
    job.init_phi(w["phi0"][0], w["phi0"][1])
    prev = job.extract()[0].astype(np.float64).ravel()
    rng = np.random.default_rng(seed)
    K = oprm["reinit_every"]
    worst, worst_full, where, reinits = 0.0, 0.0, None, 0
    for s in range(steps):
        job.step(1, w["dt"], w["interp"])
        cur, band, nb, si = job.extract()
        assert si == s + 1
        flat = cur.ravel()
        np.testing.assert_array_equal(band.ravel(),
                                      (np.abs(flat) < flat.dtype.type(gam)).astype(np.uint8))
        cur64 = flat.astype(np.float64)
        if K > 0 and (s + 1) % K == 0:
            reinits += 1
            if reinits % full_every == 0:
                if precision == "fp64":
                    ref, _ = oracle.run(prev.reshape(cur.shape), d, g, oprm, w["dt"],
                                        w["interp"], 1, step0=s)
                else:
                    ref = _reinit_from_device_step(lsr, g, prm, d, prev, cur, s, w, oprm, h)
                err = np.abs(cur64 - ref.ravel())
                worst_full = max(worst_full, float(err.max()) / h)
                want = np.abs(ref.ravel()) < gam
                sure = np.abs(np.abs(ref.ravel()) - gam) > band_margin * h
                bad = ((np.abs(cur64) < gam) != want) & sure
                if bad.any():
                    print(f"  step {s + 1}: {int(bad.sum())} band nodes differ, their values by up "
                          f"to {err[bad].max() / h:.2e} h, the state by {err.max() / h:.2e} h",
                          flush=True)
                assert not bad.any(), (s + 1, int(bad.sum()), float(err[bad].max()) / h)
        else:
            inside = np.flatnonzero(np.abs(prev) < gam)
            if len(inside):
                idx = rng.choice(inside, size=min(n_sample, len(inside)), replace=False)
                vals, _ = oracle.sl_nodes(prev.reshape(cur.shape), d, g, oprm, w["dt"],
                                          w["interp"], idx)
                e = np.abs(cur64[idx] - vals)
                if e.max() / h > worst:
                    worst = float(e.max()) / h
                    where = (s + 1, int(idx[int(e.argmax())]))
                # band membership at the sample, away from the threshold
                sure = np.abs(np.abs(vals) - gam) > band_margin * h
                assert not (((np.abs(cur64[idx]) < gam) != (np.abs(vals) < gam)) & sure).any()
            rest = rng.integers(0, len(prev), size=n_sample)
            rest = rest[np.abs(prev[rest]) >= gam]
            np.testing.assert_array_equal(cur64[rest], prev[rest])
        prev = cur64
        if (s + 1) % 100 == 0:
            print(f"  step {s + 1}: sampled max {worst:.2e} h, full checks max {worst_full:.2e} h",
                  flush=True)
    job.close()
    return worst, worst_full, where


def _reinit_from_device_step(lsr, g, prm, d, prev, cur, s, w, oprm, h):
    """For an FP32 state at a reinitialisation step: the oracle's
    reinitialisation of the device's own post-step state.  The interface
    set of the reinitialisation is decided by the signs of values near
    zero, which an FP64 step and an FP32 step may round to either side; so
    the step and the reinitialisation are checked separately, each from the
    device's own input: a twin job without reinitialisation takes the same
    step from the same state (bitwise the same post-step state), its values
    are checked against the oracle's update on the band, and the oracle
    reinitialises them on the pre-update band."""
    twin = lsr.Job(g, dict(prm, reinit_every=0))
    twin.set_distance(d)
    twin.init_phi(phi0=prev.reshape(cur.shape).astype(np.float32), step0=s)
    twin.step(1, w["dt"], w["interp"])
    post = twin.extract()[0].astype(np.float64)
    twin.close()
    prev3 = prev.reshape(cur.shape)
    band = (np.abs(prev3) < oprm["gamma"]).astype(np.uint8)
    idx = np.flatnonzero(band.ravel())[::50]
    vals, _ = oracle.sl_nodes(prev3, d, g, oprm, w["dt"], w["interp"], idx)
    assert np.abs(post.ravel()[idx] - vals).max() <= 2e-5 * h
    ref, _ = oracle.reinit(post, band, g, oprm)
    return ref


_UNION_D = {}


def union_distance():
    """The oracle's exact distance field of the 256^3 union workload, kept
    for the tests of this module."""
    if "d" not in _UNION_D:
        import time
        w = synth.workload("union3d")
        t0 = time.perf_counter()
        _UNION_D["d"] = oracle.distance(w["points"], w["grid"])
        print(f"oracle distance field of the 256^3 union: {time.perf_counter() - t0:.1f} s",
              flush=True)
    return _UNION_D["d"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_union3d_full_size(precision):
    """The 256^3 non-uniform workload (200k points, density ramp, two holes,
    WENO, dt = h/2, reinit every 10 steps), in the launch shape the bench
    times.  Every one of the 400 steps is checked against the oracle's step
    from the device's previous state on 20k sampled band nodes (1e-10 h in
    FP64; 2e-5 h in FP32, the FP32 state's own rounding, see
    test_fp32_torus3d_full_size), with every fifth reinitialisation checked
    on the whole grid.  From phi0, the scheme amplifies rounding near the
    poles of the initial sphere (tests/test_oracle_sensitivity.py): the FP64
    state stays within 1e-4 h of the oracle (band-exact away from the
    threshold) over the first 12 steps, one reinitialisation included; the
    FP32 state within 1e-4 h over the first 2 steps, and over 12 steps within
    twice the deviation that a 2^-24 relative perturbation of phi0 (the FP32
    state's resolution) makes in the oracle's own run, in the mean over the
    band and at the worst node."""
    d = union_distance()
    w = synth.workload("union3d")
    h = w["grid"]["h"]
    bar = 1e-10 if precision == "fp64" else 2e-5
    worst, worst_full, where = sampled_stepwise(w, w["steps"], d, precision)
    assert worst <= bar, (worst, where)
    assert worst_full <= bar, worst_full
    w = synth.workload("union3d", steps=12 if precision == "fp64" else 2)
    phi, band, nb, si, cnt, _ = gpu_run(w, d=d, precision=precision)
    ophi, counts, _, prm = oracle_run(w, d=d)
    e0 = check_phi(phi, ophi, h, 1e-4)
    gam = float(np.float32(prm["gamma"])) if precision == "fp32" else prm["gamma"]
    check_band(band, phi, ophi, gam, h)
    msg = (f"union3d {precision}: 400 steps sampled max {worst:.2e} h at {where}, full "
           f"reinitialisation checks max {worst_full:.2e} h; {w['steps']} steps from phi0 max "
           f"|dphi| {e0:.2e} h")
    if precision == "fp32":
        w = synth.workload("union3d", steps=12)
        phi, band, nb, si, cnt, _ = gpu_run(w, d=d, precision=precision)
        ophi, counts, _, prm = oracle_run(w, d=d)
        pphi = _perturbed_oracle(w, d, w["steps"], rel=2.0 ** -24)
        phi = phi.astype(np.float64)
        sel = (np.abs(ophi) < prm["gamma"]) | (np.abs(phi) < prm["gamma"])
        dev, env = np.abs(phi - ophi), np.abs(pphi - ophi)
        assert dev[sel].mean() <= 2 * env[sel].mean(), (dev[sel].mean() / h, env[sel].mean() / h)
        assert dev.max() <= max(2 * env.max(), 1e-4 * h), (dev.max() / h, env.max() / h)
        msg += (f"; 12 steps mean {dev[sel].mean() / h:.2e} h (envelope "
                f"{env[sel].mean() / h:.2e} h), max {dev.max() / h:.2e} h (envelope "
                f"{env.max() / h:.2e} h)")
    print(msg)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_union3d_96_whole_run(precision):
    """The union workload at 96^3 through all 400 steps: at this size the
    run does not amplify rounding (a relative 2^-24 perturbation of phi0
    leaves the oracle's end state within 1e-16 h in the mean), so the whole
    run is held to 1e-4 h of the oracle, band-exact away from the threshold,
    with the same attachment to the cloud (Err_S within 0.02 h)."""
    w = synth.workload("union3d", n=96)
    h = w["grid"]["h"]
    d = oracle.distance(w["points"], w["grid"])
    phi, band, nb, si, cnt, _ = gpu_run(w, d=d, precision=precision)
    ophi, counts, _, prm = oracle_run(w, d=d)
    e = check_phi(phi, ophi, h, 1e-4)
    gam = float(np.float32(prm["gamma"])) if precision == "fp32" else prm["gamma"]
    check_band(band, phi, ophi, gam, h)
    # nodes whose value sits at gamma to rounding stay there (c(gamma) = 0)
    # and are counted in the band or not by the last bit, step after step
    assert abs(cnt["node_updates"] - counts[0]) <= 1e-4 * counts[0]
    eg = _err_cloud(phi.astype(np.float64), w["grid"], w["points"])
    eo = _err_cloud(ophi, w["grid"], w["points"])
    assert abs(eg - eo) < 0.02 * h, (eg / h, eo / h)
    print(f"union3d 96^3 {precision}: 400 steps max |dphi| {e:.2e} h; Err_S {eg / h:.4f} h "
          f"vs {eo / h:.4f} h")


def test_torus_reaches_the_cloud():
    """Sanity of the method on the 128^3 torus workload (not parity; the
    steps are checked against the oracle above): run on to 600 steps, the
    zero level set attaches to the cloud, Err_S of eq. (errCloud) below
    0.5 h, and lies within O(h) of the closed-form torus, the mean
    |phi - SDF| over the nodes within gamma of the torus below h.  At the
    workload's 300 steps the front is still closing the torus's hole: the
    oracle's Err_S is 1.34 h there, 0.62 h at 400, 0.30 h at 500 and 0.25 h
    from 600 steps on, with delta = 0 as with delta = 1."""
    w = synth.workload("torus3d", steps=600)
    g = w["grid"]
    h = g["h"]
    phi = gpu_run(w, precision="fp32")[0].astype(np.float64)
    X = oracle.node_coords(g)
    rho = np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2) - 0.5
    sdf = (np.sqrt(rho ** 2 + X[:, 2] ** 2) - 0.2).reshape(g["n"])
    near = np.abs(sdf) < w["gamma"]
    l1 = float(np.abs(phi - sdf)[near].mean())
    es = _err_cloud(phi, g, w["points"])
    assert es < 0.5 * h and l1 < h, (es / h, l1 / h)
    print(f"torus at 600 steps: Err_S {es / h:.3f} h, mean |phi - SDF| near the surface {l1 / h:.3f} h")


# ------------------------------------------------------- reinitialisation

@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("dim", [2, 3])
def test_reinit_alone_matches_oracle(dim, precision):
    lsr = _lsr()
    n = 64 if dim == 2 else 40
    g = synth.cube_grid(dim, n)
    h = g["h"]
    X = oracle.node_coords(g)
    r = np.linalg.norm(X - 0.03, axis=1)
    phi0 = ((1.0 + 0.5 * X[:, 0]) * (r - 0.55)).reshape(g["n"])  # not a distance
    prm = oracle.default_params(dim, h)
    job = lsr.Job(g, dict(gamma=prm["gamma"], beta=prm["beta"], precision=precision), max_points=1)
    job.set_distance(np.zeros(g["n"]))
    dt = np.float64 if precision == "fp64" else np.float32
    job.init_phi(phi0=phi0.astype(dt))
    job.reinit()
    phi, band, nb, _ = job.extract()
    cnt = job.counters()
    job.close()
    pc = np.clip(phi0.astype(dt).astype(np.float64), -prm["gamma"], prm["gamma"])
    ophi, oc = oracle.reinit(pc, oracle.band_mask(pc, prm), g, prm)
    check_phi(phi, ophi, h, 1e-5)
    assert cnt["gbar"] == oc[0] and cnt["interface"] == oc[1]


# --------------------------------------------------------- edge cases

def test_empty_band_is_a_no_op():
    w = synth.workload("torus3d", n=24, steps=5)
    w["phi0"] = ("sphere", (0.0, 0.0, 0.0, 5.0))  # every node far inside: phi = -gamma
    phi, band, nb, si, cnt, _ = gpu_run(w)
    assert nb == 0 and cnt["node_updates"] == 0 and si == 5
    np.testing.assert_array_equal(phi, phi.dtype.type(-w["gamma"]))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_minimal_grid_and_band_on_the_boundary(precision):
    """n = 4 per axis: every WENO stencil is clamped and every gradient at the
    boundary is one-sided."""
    g = synth.cube_grid(3, 6)
    pts = np.array([[0.1, -0.2, 0.05], [-0.3, 0.2, 0.1], [0.5, 0.5, -0.5]])
    for n in (4, 6):
        g = synth.cube_grid(3, n)
        w = dict(grid=g, points=pts, phi0=("sphere", (0.0, 0.0, 0.0, 0.6)), interp="weno",
                 dt=0.5 * g["h"], steps=4, gamma=6 * g["h"], beta=3 * g["h"], reinit_every=2)
        phi, band, nb, _, _, _ = gpu_run(w, precision=precision)
        ophi, _, _, prm = oracle_run(w)
        check_phi(phi, ophi, g["h"], 1e-5)


@pytest.mark.parametrize("steps", [6, 16])
@pytest.mark.parametrize("dim,interp", [(3, "weno"), (3, "q1"), (2, "weno")])
def test_single_point_cloud(dim, interp, steps):
    """A cloud of one point off the grid's nodes: d is the distance to it
    (a cone with its tip between nodes).  The front shrinks toward the point,
    reinitialising on the way (6 steps), and vanishes: by 16 steps the band
    is empty and phi is +gamma everywhere."""
    g = synth.cube_grid(dim, 33)
    pts = np.array([[0.113, -0.071, 0.052][:dim]])
    w = dict(grid=g, points=pts, phi0=("sphere", (0.0, 0.0, 0.0, 0.35)), interp=interp,
             dt=0.5 * g["h"], steps=steps, gamma=6 * g["h"], beta=3 * g["h"], reinit_every=4)
    phi, band, nb, si, cnt, dgpu = gpu_run(w)
    ophi, counts, dor, prm = oracle_run(w)
    assert (np.abs(dgpu - dor) <= 4 * np.spacing(dor)).all()
    check_phi(phi, ophi, g["h"], 1e-5)
    check_band(band, phi, ophi, prm["gamma"], g["h"])
    assert si == steps and cnt["node_updates"] == counts[0]
    if steps == 16:
        assert nb == 0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_torus_initial_data_and_ragged_2d(precision):
    g = {"dim": 2, "n": (50, 77), "lo": (-1.0, -1.5), "h": 2.0 / 49}
    pts = synth.circle_cloud(300, 0.6, seed=4)
    w = dict(grid=g, points=pts, phi0=("sphere", (0.1, -0.1, 0.0, 0.8)), interp="weno",
             dt=g["h"], steps=20, gamma=6 * g["h"], beta=3 * g["h"], reinit_every=1)
    phi, band, nb, _, _, _ = gpu_run(w, precision=precision)
    ophi, _, _, prm = oracle_run(w)
    check_phi(phi, ophi, g["h"], 1e-4)
    # Torus phi0 on a grid with a node at its centre: the nodes of its axis
    # and of its plane of symmetry sit on frame ties and on the cone points of
    # phi0 and d.  FP64 state: 1e-4 h.  FP32 state: the oracle itself moves by
    # ~3e-2 h when phi0 is perturbed at FP32 resolution, so the bar is twice
    # that envelope (floored at 1e-4 h).
    w3 = synth.workload("torus3d", n=33, steps=6)
    w3["phi0"] = ("torus", (0.0, 0.0, 0.0, 0.5, 0.25))
    h3 = w3["grid"]["h"]
    phi, band, nb, _, _, _ = gpu_run(w3, precision=precision)
    ophi, _, d3, prm = oracle_run(w3)
    if precision == "fp64":
        check_phi(phi, ophi, h3, 1e-4)
    else:
        env = np.abs(_perturbed_oracle(w3, d3, w3["steps"], rel=2.0 ** -24) - ophi).max()
        check_phi(phi, ophi, h3, max(1e-4, 2 * env / h3))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_fallback_and_array_initial_data(precision):
    """A flat plateau inside the band takes the degenerate-gradient branch."""
    g = synth.cube_grid(3, 24)
    h = g["h"]
    X = oracle.node_coords(g)
    # plateaus at -h/2 (inside the band) and 5h (clear of the threshold gamma = 6h)
    phi0 = np.clip(np.linalg.norm(X, axis=1) - 0.5, -0.5 * h, 5 * h).reshape(g["n"])
    w = dict(grid=g, points=synth.torus_cloud(2000, 0.5, 0.2, 0.0, seed=3),
             phi0=("array", phi0), interp="weno", dt=0.5 * h, steps=3,
             gamma=6 * h, beta=3 * h, reinit_every=0)
    phi, band, nb, _, cnt, _ = gpu_run(w, precision=precision)
    ophi, counts, _, prm = oracle_run(w)
    check_phi(phi, ophi, h, 1e-5)
    assert cnt["fallbacks"] == counts[1] and counts[1] > 0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_restart_is_bitwise_identical(precision):
    w = synth.workload("torus3d", n=40, steps=20)
    full, _, _, _, _, _ = gpu_run(w, precision=precision)
    half, _, _, _, _, _ = gpu_run(w, steps=7, precision=precision)
    w2 = dict(w)
    w2["phi0"] = ("array", half)
    rest, _, _, si, _, _ = gpu_run(w2, steps=13, step0=7, precision=precision)
    assert si == 20
    np.testing.assert_array_equal(full, rest)


def test_errors_leave_the_job_usable():
    lsr = _lsr()
    w = synth.workload("torus3d", n=24)
    job = lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"]), max_points=len(w["points"]))
    with pytest.raises(lsr.LsrError) as e:
        job.step(1, w["dt"], "weno")
    assert e.value.status == lsr.LSR_E_STATE
    job.load_cloud(w["points"])
    d1 = job.distance()
    bad = w["points"].copy()
    bad[5, 1] = np.nan
    with pytest.raises(lsr.LsrError) as e:
        job.load_cloud(bad)
    assert e.value.status == lsr.LSR_E_INVALID
    bad = w["points"].copy()
    bad[7, 0] = 1.5
    with pytest.raises(lsr.LsrError):
        job.load_cloud(bad)
    np.testing.assert_array_equal(job.distance(), d1)
    phi0 = np.zeros(w["grid"]["n"], np.float32)
    phi0[1, 2, 3] = np.inf
    with pytest.raises(lsr.LsrError):
        job.init_phi(phi0=phi0)
    job.init_phi("sphere", (0, 0, 0, 0.9))
    job.step(2, w["dt"], "weno")
    assert job.extract()[3] == 2
    job.close()


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,interp", [("torus3d", "weno"), ("torus3d", "q1"),
                                         ("circle2d", "weno")])
def test_launch_shape_does_not_change_results(name, interp, precision):
    """One lane per node and one lane per foot point read the same values and
    add the foot values in the same order: bitwise equal results, whatever
    the persistent grid (1 block per CU leaves most chunks of the band to a
    second round of the blocks).  12 steps cross a reinitialisation."""
    lsr = _lsr()
    w = synth.workload(name, n=40 if name == "torus3d" else 96, steps=12)
    w["interp"] = interp
    fp = 4 if w["grid"]["dim"] == 3 else 2
    shapes = [(1, 8), (fp, 8), (1, 2), (fp, 1)]
    out = []
    for lanes, bpc in shapes:
        oprm = oracle_params(w)
        prm = {k: oprm[k] for k in ("gamma", "beta", "reinit_every", "reinit_iters")}
        prm["precision"] = precision
        job = lsr.Job(w["grid"], prm, max_points=len(w["points"]))
        job.set_launch(lanes, bpc)
        job.load_cloud(w["points"])
        job.init_phi(w["phi0"][0], w["phi0"][1])
        job.step(w["steps"], w["dt"], interp)
        out.append(job.extract()[0])
        job.close()
    for o in out[1:]:
        np.testing.assert_array_equal(out[0], o)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_launch_shapes_on_a_ragged_grid(precision):
    """Ragged extents (no axis a multiple of a brick): the list builds scan
    partial bricks and slots, the chunked band lists end in partial chunks;
    every launch shape gives the same result and the same work counts."""
    lsr = _lsr()
    g = {"dim": 3, "n": (23, 41, 30), "lo": (-0.6, -1.0, -0.75), "h": 0.05}
    pts = synth.torus_cloud(3000, 0.45, 0.18, 0.0, seed=9)
    pts = pts[np.all(np.abs(pts) < [0.5, 0.9, 0.7], axis=1)]
    out = []
    for lanes, bpc in ((1, 8), (4, 8), (1, 1)):
        job = lsr.Job(g, dict(gamma=0.3, beta=0.15, reinit_every=4, precision=precision),
                      max_points=len(pts))
        job.set_launch(lanes, bpc)
        job.load_cloud(pts)
        job.init_phi("sphere", (0.0123, 0.0571, -0.0087, 0.55))
        job.step(9, 0.025, "weno")
        out.append((job.extract()[0], job.counters()))
        job.close()
    for o in out[1:]:
        np.testing.assert_array_equal(out[0][0], o[0])
        assert out[0][1] == o[1]
