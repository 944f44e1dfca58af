"""ctypes binding of ``include/lsr.h`` (liblsr.so, the HIP library).

The ``lsr_*`` functions mirror the C entry points one to one and only
marshal arguments; every step of the solver runs in the library's kernels.
:class:`Job` is a convenience owner of a job: it allocates the workspace as a
torch uint8 tensor, passes torch's current HIP stream and converts inputs and
outputs.  PyTorch is used for device memory and streams only.

There is no CPU fallback: if the library is missing, importing the binding
works but the first call raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblsr.so")

LSR_OK, LSR_E_INVALID, LSR_E_NOMEM, LSR_E_DEVICE, LSR_E_STATE, LSR_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
LSR_Q1, LSR_WENO = 0, 1
LSR_PHI_ARRAY, LSR_PHI_SPHERE, LSR_PHI_TORUS = 0, 1, 2
LSR_FP32, LSR_FP64 = 0, 1
COUNTER_NAMES = ["node_updates", "fallbacks", "frame0", "reinits", "gbar", "interface", "steps"]

EXPORTED = [
    "lsr_params_default", "lsr_workspace_bytes", "lsr_create", "lsr_load_cloud",
    "lsr_set_distance", "lsr_get_distance", "lsr_init_phi", "lsr_step", "lsr_reinit",
    "lsr_extract", "lsr_energy", "lsr_energy_stop", "lsr_run_to_steady", "lsr_cloud_spacing",
    "lsr_counters",
    "lsr_destroy", "lsr_batch_workspace_bytes", "lsr_batch_create",
    "lsr_batch_add", "lsr_batch_remove", "lsr_batch_step", "lsr_batch_set_launch",
    "lsr_batch_tune", "lsr_batch_destroy", "lsr_batch_set_graphs", "lsr_batch_set_streams",
    "lsr_set_launch",
    "lsr_set_graphs", "lsr_graph_counts", "lsr_profile_enable",
    "lsr_profile_read", "lsr_last_error", "lsr_load_cloud_approx", "lsr_init_phi_cloud",
    "lsr_init_phi_resample", "lsr_schedule_run", "lsr_set_tune_cache", "lsr_energy_noalloc",
]


class LsrGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("h", ctypes.c_double)]


class LsrParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("delta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("grad_C", ctypes.c_double), ("grad_alpha", ctypes.c_double),
                ("reinit_every", ctypes.c_int32), ("reinit_iters", ctypes.c_int32),
                ("reinit_dtau", ctypes.c_double), ("interface_floor", ctypes.c_double),
                ("precision", ctypes.c_int32)]


class LsrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lsr status {status}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p


def load():
    """Open liblsr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        GP, PP = ctypes.POINTER(LsrGrid), ctypes.POINTER(LsrParams)
        I64P = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "lsr_params_default": [ctypes.c_int32, ctypes.c_double, PP],
            "lsr_workspace_bytes": [GP, PP, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
            "lsr_create": [GP, PP, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
            "lsr_load_cloud": [_P, _P, ctypes.c_int64],
            "lsr_load_cloud_approx": [_P, _P, ctypes.c_int64],
            "lsr_init_phi_cloud": [_P, ctypes.c_double, ctypes.c_int64],
            "lsr_init_phi_resample": [_P, _P, ctypes.c_int, ctypes.c_int64],
            "lsr_schedule_run": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                                 GP, PP, ctypes.POINTER(ctypes.c_double)],
            "lsr_set_distance": [_P, _P],
            "lsr_get_distance": [_P, _P],
            "lsr_init_phi": [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int64],
            "lsr_step": [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int],
            "lsr_reinit": [_P],
            "lsr_extract": [_P, _P, _P, I64P, I64P],
            "lsr_energy": [_P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
            "lsr_cloud_spacing": [_P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)],
            "lsr_energy_stop": [ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_double],
            "lsr_run_to_steady": [_P, ctypes.c_double, ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32)],
            "lsr_counters": [_P, I64P, ctypes.c_int32],
            "lsr_destroy": [_P],
            "lsr_batch_workspace_bytes": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_size_t)],
            "lsr_batch_create": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t,
                                 _P, ctypes.POINTER(_P)],
            "lsr_batch_add": [_P, _P, ctypes.c_double, ctypes.c_int],
            "lsr_batch_remove": [_P, _P],
            "lsr_batch_step": [_P, ctypes.c_int32],
            "lsr_batch_set_launch": [_P, ctypes.c_int32, ctypes.c_int32],
            "lsr_batch_tune": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double)],
            "lsr_batch_destroy": [_P],
            "lsr_set_tune_cache": [ctypes.c_char_p],
            "lsr_energy_noalloc": [GP, ctypes.c_int32, _P, _P, ctypes.c_double, ctypes.c_int32, _P,
                                   _P],
            "lsr_profile_enable": [_P, ctypes.c_int32, ctypes.c_int32],
            "lsr_set_launch": [_P, ctypes.c_int32, ctypes.c_int32],
            "lsr_set_graphs": [_P, ctypes.c_int32],
            "lsr_batch_set_graphs": [_P, ctypes.c_int32],
            "lsr_batch_set_streams": [_P, ctypes.c_int32],
            "lsr_graph_counts": [_P, _P, I64P, I64P],
            "lsr_profile_read": [_P, ctypes.POINTER(ctypes.c_double), I64P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.lsr_last_error.argtypes = []
        lib.lsr_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def lsr_last_error():
    return load().lsr_last_error().decode()


def _check(status):
    if status != LSR_OK:
        raise LsrError(status, lsr_last_error())


def make_grid(grid):
    g = LsrGrid()
    g.dim = int(grid["dim"])
    n = list(grid["n"]) + [1] * (3 - len(grid["n"]))
    lo = list(grid["lo"]) + [0.0] * (3 - len(grid["lo"]))
    for a in range(3):
        g.n[a] = int(n[a])
        g.lo[a] = float(lo[a])
    g.h = float(grid["h"])
    return g


# ------------------------------------------------------- C entry points

def lsr_params_default(dim, h):
    p = LsrParams()
    _check(load().lsr_params_default(int(dim), float(h), ctypes.byref(p)))
    return p


def lsr_workspace_bytes(grid, params, max_points):
    out = ctypes.c_size_t()
    _check(load().lsr_workspace_bytes(ctypes.byref(grid), ctypes.byref(params) if params else None,
                                      int(max_points), ctypes.byref(out)))
    return out.value


def lsr_create(grid, params, ws_ptr, ws_bytes, stream_ptr):
    h = _P()
    _check(load().lsr_create(ctypes.byref(grid), ctypes.byref(params), _P(ws_ptr), int(ws_bytes),
                             _P(stream_ptr), ctypes.byref(h)))
    return h


def lsr_load_cloud(job, xyz_ptr, n):
    _check(load().lsr_load_cloud(job, _P(xyz_ptr), int(n)))


def lsr_load_cloud_approx(job, xyz_ptr, n):
    _check(load().lsr_load_cloud_approx(job, _P(xyz_ptr), int(n)))


def lsr_init_phi_cloud(job, gamma_s, step0=0):
    _check(load().lsr_init_phi_cloud(job, float(gamma_s), int(step0)))


def lsr_init_phi_resample(job, coarse, interp, step0=0):
    _check(load().lsr_init_phi_resample(job, coarse, int(interp), int(step0)))


def lsr_schedule_run(r, dim, box_lo, box_hi, h_s, k_s=2.0):
    """(grid, params, dt) of run r of the coarse-to-fine schedule."""
    lo = (ctypes.c_double * 3)(*(list(box_lo) + [0.0] * (3 - len(box_lo))))
    hi = (ctypes.c_double * 3)(*(list(box_hi) + [0.0] * (3 - len(box_hi))))
    g, p, dt = LsrGrid(), LsrParams(), ctypes.c_double()
    _check(load().lsr_schedule_run(int(r), int(dim), lo, hi, float(h_s), float(k_s),
                                   ctypes.byref(g), ctypes.byref(p), ctypes.byref(dt)))
    return g, p, dt.value


def lsr_set_distance(job, d_ptr):
    _check(load().lsr_set_distance(job, _P(d_ptr)))


def lsr_get_distance(job, out_ptr):
    _check(load().lsr_get_distance(job, _P(out_ptr)))


def lsr_init_phi(job, phi_ptr, kind, args, step0):
    a = (ctypes.c_double * 8)(*([float(x) for x in (args or [])] + [0.0] * (8 - len(args or []))))
    _check(load().lsr_init_phi(job, _P(phi_ptr) if phi_ptr else None, int(kind), a, int(step0)))


def lsr_step(job, n_steps, dt, interp):
    _check(load().lsr_step(job, int(n_steps), float(dt), int(interp)))


def lsr_reinit(job):
    _check(load().lsr_reinit(job))


def lsr_extract(job, phi_ptr, band_ptr, want_count=True):
    nb = ctypes.c_int64(-1)
    si = ctypes.c_int64(-1)
    _check(load().lsr_extract(job, _P(phi_ptr) if phi_ptr else None,
                              _P(band_ptr) if band_ptr else None,
                              ctypes.byref(nb) if want_count else None, ctypes.byref(si)))
    return nb.value, si.value


def lsr_energy(job, p, R=5):
    out = ctypes.c_double(0.0)
    _check(load().lsr_energy(job, float(p), int(R), ctypes.byref(out)))
    return out.value


def lsr_cloud_spacing(job, sample_ptr, n_sample):
    out = ctypes.c_double(0.0)
    _check(load().lsr_cloud_spacing(job, _P(sample_ptr), int(n_sample), ctypes.byref(out)))
    return out.value


def lsr_energy_stop(energies, n, min_steps=10, max_steps=100, tol=1e-4):
    e = (ctypes.c_double * max(len(energies), 1))(*energies)
    return load().lsr_energy_stop(e, int(n), int(min_steps), int(max_steps), float(tol))


def lsr_run_to_steady(job, dt, interp, min_steps=10, max_steps=100, tol=1e-4):
    e = (ctypes.c_double * (max_steps + 1))()
    n = ctypes.c_int32(0)
    _check(load().lsr_run_to_steady(job, float(dt), int(interp), int(min_steps), int(max_steps),
                                    float(tol), e, ctypes.byref(n)))
    return n.value, list(e[: n.value + 1])


def lsr_counters(job):
    out = (ctypes.c_int64 * len(COUNTER_NAMES))()
    _check(load().lsr_counters(job, out, len(COUNTER_NAMES)))
    return dict(zip(COUNTER_NAMES, list(out)))


def lsr_destroy(job):
    _check(load().lsr_destroy(job))


def lsr_batch_workspace_bytes(max_jobs, group_steps, max_reinit_iters):
    out = ctypes.c_size_t()
    _check(load().lsr_batch_workspace_bytes(int(max_jobs), int(group_steps), int(max_reinit_iters),
                                            ctypes.byref(out)))
    return out.value


def lsr_batch_create(max_jobs, group_steps, max_reinit_iters, ws_ptr, ws_bytes, stream_ptr):
    h = _P()
    _check(load().lsr_batch_create(int(max_jobs), int(group_steps), int(max_reinit_iters),
                                   _P(ws_ptr), int(ws_bytes), _P(stream_ptr), ctypes.byref(h)))
    return h


def lsr_batch_add(batch, job, dt, interp):
    _check(load().lsr_batch_add(batch, job, float(dt), int(interp)))


def lsr_batch_remove(batch, job):
    _check(load().lsr_batch_remove(batch, job))


def lsr_batch_step(batch, n_steps):
    _check(load().lsr_batch_step(batch, int(n_steps)))


def lsr_batch_set_launch(batch, lanes, blocks_per_cu):
    _check(load().lsr_batch_set_launch(batch, int(lanes), int(blocks_per_cu)))


def lsr_batch_tune(batch):
    lanes, bpc, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().lsr_batch_tune(batch, ctypes.byref(lanes), ctypes.byref(bpc), ctypes.byref(ms)))
    return lanes.value, bpc.value, ms.value


def lsr_energy_noalloc(grid, precision, phi_ptr, d_ptr, p, R, out_ptr, stream_ptr):
    """E_p of device fields into the device double at out_ptr, with no job,
    workspace or allocation (see lsr.h)."""
    return load().lsr_energy_noalloc(ctypes.byref(grid), int(precision), _P(phi_ptr), _P(d_ptr),
                                     float(p), int(R), _P(out_ptr), _P(stream_ptr))


def lsr_set_tune_cache(path):
    _check(load().lsr_set_tune_cache(path.encode() if path else None))


def lsr_batch_destroy(batch):
    _check(load().lsr_batch_destroy(batch))


def lsr_set_launch(job, lanes, blocks_per_cu):
    _check(load().lsr_set_launch(job, int(lanes), int(blocks_per_cu)))


def lsr_set_graphs(job, enable):
    _check(load().lsr_set_graphs(job, int(bool(enable))))


def lsr_batch_set_graphs(batch, enable):
    _check(load().lsr_batch_set_graphs(batch, int(bool(enable))))


def lsr_batch_set_streams(batch, n_streams):
    _check(load().lsr_batch_set_streams(batch, int(n_streams)))


def lsr_graph_counts(job=None, batch=None):
    """(graphs recorded, graph replays) of a job's or a batch's step loop."""
    c, r = ctypes.c_int64(), ctypes.c_int64()
    _check(load().lsr_graph_counts(job, batch, ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


def lsr_profile_enable(job, enable, max_launches=4096):
    _check(load().lsr_profile_enable(job, int(bool(enable)), int(max_launches)))


def lsr_profile_read(job):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().lsr_profile_read(job, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------ convenience

def interp_code(name):
    return {"q1": LSR_Q1, "weno": LSR_WENO}[name]


class Job:
    """One reconstruction on the current device.

    grid: {"dim", "n", "lo", "h"}; params: overrides of lsr_params_default
    (``precision``: "fp32" or "fp64" also accepted); max_points: largest
    cloud to be loaded; stream: a torch.cuda.Stream (default: the current
    stream)."""

    def __init__(self, grid, params=None, max_points=0, stream=None):
        import torch
        self.torch = torch
        self.grid_dict = dict(grid)
        self.grid = make_grid(grid)
        self.params = lsr_params_default(self.grid.dim, self.grid.h)
        params = dict(params or {})
        if isinstance(params.get("precision"), str):
            params["precision"] = {"fp32": LSR_FP32, "fp64": LSR_FP64}[params["precision"]]
        for k, v in params.items():
            setattr(self.params, k, v)
        if "reinit_iters" not in params and ("gamma" in params or "reinit_dtau" in params):
            # the default iteration count follows the band width: ceil((gamma + h)/dtau)
            p = self.params
            p.reinit_iters = int(np.ceil((p.gamma + self.grid.h) / p.reinit_dtau - 1e-9))
        self.shape = tuple(int(v) for v in grid["n"][: self.grid.dim])
        self.nodes = int(np.prod(self.shape))
        self.fp64 = self.params.precision == LSR_FP64
        self.dtype = torch.float64 if self.fp64 else torch.float32
        self.ws_bytes = lsr_workspace_bytes(self.grid, self.params, max_points)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.stream.device)
        self.handle = lsr_create(self.grid, self.params, self.ws.data_ptr(), self.ws_bytes,
                                 self.stream.cuda_stream)

    def _dev(self, x, dtype):
        t = self.torch.as_tensor(np.ascontiguousarray(x) if isinstance(x, np.ndarray) else x)
        return t.to(device=self.stream.device, dtype=dtype).contiguous()

    def load_cloud(self, points, approx=False):
        """The cloud and its distance field: exact, or (approx) the paper's
        approximation of Section 3.4."""
        pts = self._dev(points, self.torch.float64)
        self.torch.cuda.current_stream().synchronize()  # the copy, before the job's stream reads it
        (lsr_load_cloud_approx if approx else lsr_load_cloud)(self.handle, pts.data_ptr(),
                                                             pts.shape[0])

    def init_phi_cloud(self, gamma_s, step0=0):
        """phi0 from the loaded distance field (Section 3.6)."""
        lsr_init_phi_cloud(self.handle, gamma_s, step0)

    def init_phi_resample(self, coarse, interp, step0=0):
        """phi0 = the coarser job's phi interpolated onto this grid (Section 4)."""
        lsr_init_phi_resample(self.handle, coarse.handle,
                              interp_code(interp) if isinstance(interp, str) else interp, step0)

    def set_distance(self, d):
        dd = self._dev(d, self.torch.float64)
        self._keep = dd
        lsr_set_distance(self.handle, dd.data_ptr())

    def distance(self):
        out = self.torch.empty(self.nodes, dtype=self.torch.float64, device=self.stream.device)
        lsr_get_distance(self.handle, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy().reshape(self.shape)

    def init_phi(self, kind="sphere", args=(), phi0=None, step0=0):
        if phi0 is not None:
            t = self._dev(phi0, self.dtype)
            self._keep = t
            lsr_init_phi(self.handle, t.data_ptr(), LSR_PHI_ARRAY, [], step0)
        else:
            k = {"sphere": LSR_PHI_SPHERE, "torus": LSR_PHI_TORUS}[kind]
            lsr_init_phi(self.handle, None, k, list(args), step0)

    def step(self, n_steps, dt, interp):
        lsr_step(self.handle, n_steps, dt, interp_code(interp) if isinstance(interp, str) else interp)

    def reinit(self):
        lsr_reinit(self.handle)

    def extract_device(self):
        phi = self.torch.empty(self.nodes, dtype=self.dtype, device=self.stream.device)
        band = self.torch.empty(self.nodes, dtype=self.torch.uint8, device=self.stream.device)
        nb, si = lsr_extract(self.handle, phi.data_ptr(), band.data_ptr(), want_count=True)
        return phi.view(self.shape), band.view(self.shape), nb, si

    def extract(self):
        phi, band, nb, si = self.extract_device()
        self.stream.synchronize()
        return phi.cpu().numpy(), band.cpu().numpy(), nb, si

    def run_to_steady(self, dt, interp, min_steps=10, max_steps=100, tol=1e-4):
        """Steps until the energy test of eq. (deltaEn) stops the run; returns
        (steps taken, [E_2(phi^0), ..., E_2(phi^n)])."""
        code = interp_code(interp) if isinstance(interp, str) else interp
        return lsr_run_to_steady(self.handle, dt, code, min_steps, max_steps, tol)

    def cloud_spacing(self, sample):
        """h_S of the loaded cloud over the sampled point indices (Section 4);
        synchronises the stream."""
        t = self._dev(np.asarray(sample, dtype=np.int64), self.torch.int64)
        self.torch.cuda.current_stream().synchronize()  # the copy, before the job's stream reads it
        return lsr_cloud_spacing(self.handle, t.data_ptr(), t.numel())

    def energy(self, p, R=5):
        """E_p of the current phi (Section 3.5); synchronises the stream."""
        return lsr_energy(self.handle, p, R)

    def counters(self):
        return lsr_counters(self.handle)

    def set_launch(self, lanes, blocks_per_cu=8):
        lsr_set_launch(self.handle, lanes, blocks_per_cu)

    def set_graphs(self, enable):
        lsr_set_graphs(self.handle, enable)

    def graph_counts(self):
        return lsr_graph_counts(job=self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            lsr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched stepping of Jobs on one stream (see lsr_batch_* in lsr.h)."""

    def __init__(self, max_jobs, group_steps=64, max_reinit_iters=32, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws_bytes = lsr_batch_workspace_bytes(max_jobs, group_steps, max_reinit_iters)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.stream.device)
        self.handle = lsr_batch_create(max_jobs, group_steps, max_reinit_iters, self.ws.data_ptr(),
                                       self.ws_bytes, self.stream.cuda_stream)
        self.members = []

    def add(self, job, dt, interp):
        lsr_batch_add(self.handle, job.handle, dt,
                      interp_code(interp) if isinstance(interp, str) else interp)
        job.stream_saved = job.stream
        job.stream = self.stream
        self.members.append(job)

    def remove(self, job):
        lsr_batch_remove(self.handle, job.handle)
        job.stream = job.stream_saved
        self.members.remove(job)

    def step(self, n_steps):
        lsr_batch_step(self.handle, n_steps)

    def set_launch(self, lanes, blocks_per_cu):
        lsr_batch_set_launch(self.handle, lanes, blocks_per_cu)

    def set_graphs(self, enable):
        lsr_batch_set_graphs(self.handle, enable)

    def set_streams(self, n_streams):
        lsr_batch_set_streams(self.handle, n_streams)

    def graph_counts(self):
        return lsr_graph_counts(batch=self.handle)

    def tune(self):
        return lsr_batch_tune(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            for job in list(self.members):
                self.remove(job)
            lsr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
