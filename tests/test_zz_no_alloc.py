"""lsr_energy_noalloc (the entry point for callers that cannot allocate)
against lsr_energy on the same fields, through the C ABI: two calls in a
row, the second on a smaller grid, each within 1e-12 relative of the
job's own energy; and the argument checks.  Collected last (its name) and
also run alone in a fresh process."""
import ctypes

import numpy as np
import pytest

from paper_2410_22205_amd import synth

pytestmark = pytest.mark.gpu


def _fn():
    """The C entry point itself, through the binding's ctypes signature."""
    from paper_2410_22205_amd import lsr
    return lsr, lsr.load().lsr_energy_noalloc


def _case(name, n, steps, precision):
    import torch
    lsr, f = _fn()
    w = synth.workload(name, n=n, steps=steps)
    job = lsr.Job(w["grid"], dict(gamma=w["gamma"], beta=w["beta"],
                                  reinit_every=w["reinit_every"], precision=precision),
                  max_points=len(w["points"]))
    job.load_cloud(w["points"])
    job.init_phi(w["phi0"][0], w["phi0"][1])
    job.step(w["steps"], w["dt"], w["interp"])
    want = job.energy(2.0)
    phi = job.extract_device()[0].contiguous()
    d = torch.empty(job.nodes, dtype=torch.float64, device="cuda")
    lsr.lsr_get_distance(job.handle, d.data_ptr())
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    job.stream.synchronize()
    st = f(ctypes.byref(job.grid), lsr.LSR_FP64 if precision == "fp64" else lsr.LSR_FP32,
           phi.data_ptr(), d.data_ptr(), 2.0, 5, out.data_ptr(),
           torch.cuda.current_stream().cuda_stream)
    assert st == lsr.LSR_OK, lsr.lsr_last_error()
    torch.cuda.synchronize()
    got = float(out.item())
    job.close()
    return got, want


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_energy_equals_job_energy(precision):
    # the job sums the same terms over a list of its front cells, in another
    # order: equal to rounding
    got, want = _case("torus3d", 48, 12, precision)
    assert want > 0 and abs(got - want) <= 1e-12 * want
    got, want = _case("circle2d", 64, 5, precision)  # a second, smaller call
    assert want > 0 and abs(got - want) <= 1e-12 * want


def test_noalloc_energy_rejects_bad_arguments():
    import torch
    lsr, f = _fn()
    g = lsr.make_grid({"dim": 3, "n": (4096, 4096, 300), "lo": (0, 0, 0), "h": 0.1})
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert f(ctypes.byref(g), lsr.LSR_FP64, x.data_ptr(), x.data_ptr(), 2.0, 5, x.data_ptr(),
             None) == lsr.LSR_E_UNSUPPORTED
    g = lsr.make_grid({"dim": 3, "n": (8, 8, 8), "lo": (0, 0, 0), "h": 0.1})
    assert f(ctypes.byref(g), 7, x.data_ptr(), x.data_ptr(), 2.0, 5, x.data_ptr(),
             None) == lsr.LSR_E_INVALID
    assert f(ctypes.byref(g), lsr.LSR_FP64, x.data_ptr(), x.data_ptr(), 2.0, 0, x.data_ptr(),
             None) == lsr.LSR_E_INVALID
    assert f(ctypes.byref(g), lsr.LSR_FP64, None, x.data_ptr(), 2.0, 5, x.data_ptr(),
             None) == lsr.LSR_E_INVALID
