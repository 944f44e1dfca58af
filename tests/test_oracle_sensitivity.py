"""A property of the scheme, pinned on the oracle: on the 128^3 torus workload
the update is unstable to rounding where the front meets the torus axis (the
distance field has a cone point there, every point of the inner ring being
equidistant), so a one-ulp perturbation of phi0 grows to a visible difference
within a few tens of steps, while on the 48^3 grid it stays at rounding level.
On the union workload the growth sits at the poles of the initial sphere on
the y axis, where the tangent frame of eq. (sigma3d) is built from the small
pair (d1 phi, d3 phi) and turns with any change of it.
This is why whole-run comparisons on these workloads are made stepwise and
against the oracle's own perturbation envelope rather than at a fixed
tolerance."""
import numpy as np
import pytest

import oracle
from paper_2410_22205_amd import synth


def _pair(n, steps, name="torus3d", where=False):
    w = synth.workload(name, n=n)
    g, h = w["grid"], w["grid"]["h"]
    prm = oracle.default_params(3, h, gamma=w["gamma"], beta=w["beta"], reinit_every=10)
    d = oracle.distance(w["points"], g)
    phi = oracle.init_phi(g, "sphere", w["phi0"][1], prm["gamma"])
    rng = np.random.default_rng(1)
    band = np.abs(phi) < prm["gamma"]
    pert = np.where(band, phi * (1 + rng.choice([-1.0, 1.0], phi.shape) * 2.0 ** -52), phi)
    a, _ = oracle.run(phi, d, g, prm, w["dt"], "weno", steps)
    b, _ = oracle.run(pert, d, g, prm, w["dt"], "weno", steps)
    e = np.abs(a - b)
    if where:
        return e.max() / h, oracle.node_coords(g)[int(e.argmax())]
    return e.max() / h, np.abs(pert - phi).max() / h


@pytest.mark.slow
def test_one_ulp_grows_to_visible_difference_at_128():
    diff, p0 = _pair(128, 35)
    assert p0 < 1e-14
    assert diff > 1e-3, diff


def test_one_ulp_stays_at_rounding_level_at_48():
    diff, p0 = _pair(48, 60)
    assert diff < 1e-10, diff


@pytest.mark.slow
def test_one_ulp_grows_at_the_frame_poles_on_the_union():
    diff, x = _pair(96, 40, name="union3d", where=True)
    assert diff > 1e-2, diff
    assert np.hypot(x[0], x[2]) < 0.25 and abs(x[1]) > 0.5, x  # next to the y axis
