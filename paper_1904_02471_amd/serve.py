"""ctypes binding of the lb_server_* C ABI (continuous batching of many
simulations), plus a trace driver that submits requests at their arrival
times and collects results with their latencies.

Argument marshalling only; the batching, admission and stepping run in
liblbm.so."""
import ctypes
import time

import numpy as np

from . import lb

_lib = lb._lib
_dp = ctypes.POINTER(ctypes.c_double)


class Request(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("Nx", ctypes.c_int), ("Ny", ctypes.c_int),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("ds", ctypes.c_double), ("N", ctypes.c_int),
                ("rho", _dp), ("ux", _dp), ("uy", _dp),
                ("ax", _dp), ("ay", _dp), ("bx", _dp), ("by", _dp),
                ("nsteps", ctypes.c_int), ("sample_every", ctypes.c_int), ("tag", ctypes.c_uint64),
                ("decay_k2", ctypes.c_double), ("decay_omega", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int),
                ("nsamples", ctypes.c_int), ("samples", _dp),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("nu_app", ctypes.c_double)]


_lib.lb_server_create.restype = ctypes.c_void_p
_lib.lb_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
_lib.lb_server_submit.restype = ctypes.c_int
_lib.lb_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
_lib.lb_server_poll.restype = ctypes.c_int
_lib.lb_server_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(Result), ctypes.c_int, ctypes.c_int]
_lib.lb_server_release.restype = None
_lib.lb_server_release.argtypes = [ctypes.c_void_p, ctypes.POINTER(Result)]
_lib.lb_server_clock.restype = ctypes.c_double
_lib.lb_server_clock.argtypes = [ctypes.c_void_p]
_lib.lb_server_stats.restype = ctypes.c_int
_lib.lb_server_stats.argtypes = [ctypes.c_void_p, _dp]
_lib.lb_server_configure.restype = ctypes.c_int
_lib.lb_server_configure.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
_lib.lb_server_set_node_limit.restype = ctypes.c_int
_lib.lb_server_set_node_limit.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
_lib.lb_server_set_policy.restype = ctypes.c_int
_lib.lb_server_set_policy.argtypes = [ctypes.c_void_p, ctypes.c_int]
ADMIT_ARRIVAL, ADMIT_SHORTEST = 0, 1
_lib.lb_fit_decay.restype = ctypes.c_int
_lib.lb_fit_decay.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_double, _dp]
_lib.lb_server_destroy.restype = None
_lib.lb_server_destroy.argtypes = [ctypes.c_void_p]


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


class Server:
    """Python handle of an lb_server.  Keeps the host arrays of every
    submitted request alive until its result is polled."""

    def __init__(self, hbm_budget_bytes=64 << 30, max_slots=512, chunk_steps=32, use_graphs=True, tune_tiles=True,
                 node_limit=0, policy=0):
        h = _lib.lb_server_create(int(hbm_budget_bytes), int(max_slots), int(chunk_steps))
        if not h:
            raise lb.LBError(lb.lb_last_error(), "lb_server_create")
        self._h = h
        self._keep = {}
        rc = _lib.lb_server_configure(h, int(bool(use_graphs)), int(bool(tune_tiles)))
        if rc != lb.LB_OK:
            raise lb.LBError(rc, "lb_server_configure")
        rc = _lib.lb_server_set_node_limit(h, int(node_limit))
        if rc != lb.LB_OK:
            raise lb.LBError(rc, "lb_server_set_node_limit")
        rc = _lib.lb_server_set_policy(h, int(policy))
        if rc != lb.LB_OK:
            raise lb.LBError(rc, "lb_server_set_policy")

    def submit(self, model, Nx, Ny, tau, dt, ds, N, rho, ux, uy, nsteps, sample_every, probe=None, tag=0,
               decay_k2=0.0, decay_omega=0.0):
        shp = (Ny, Nx)
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shp)) for a in (rho, ux, uy)]
        pr = [None] * 4
        if probe is not None:
            pr = [np.ascontiguousarray(np.asarray(v, np.float64)) for v in probe]
        r = Request(int(model), int(Nx), int(Ny), float(tau), float(dt), float(ds), int(N),
                    _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), _ptr(pr[0]), _ptr(pr[1]), _ptr(pr[2]), _ptr(pr[3]),
                    int(nsteps), int(sample_every), int(tag), float(decay_k2), float(decay_omega))
        rid = ctypes.c_uint64(0)
        rc = _lib.lb_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if rc != lb.LB_OK:
            raise lb.LBError(rc, "lb_server_submit")
        self._keep[rid.value] = (arrs, pr)
        return rid.value

    def poll(self, max_results=64, timeout_us=0):
        """List of dicts {id, tag, status, samples (n x 6), t_submit, t_admit, t_finish}."""
        buf = (Result * int(max_results))()
        n = _lib.lb_server_poll(self._h, buf, int(max_results), int(timeout_us))
        if n < 0:
            raise lb.LBError(n, "lb_server_poll")
        out = []
        for i in range(n):
            r = buf[i]
            samples = np.ctypeslib.as_array(r.samples, shape=(r.nsamples, 6)).copy() if r.nsamples else np.zeros((0, 6))
            out.append({"id": r.id, "tag": r.tag, "status": r.status, "samples": samples,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_finish": r.t_finish,
                        "nu_app": r.nu_app})
            _lib.lb_server_release(self._h, ctypes.byref(r))
            self._keep.pop(r.id, None)
        return out

    def clock(self):
        return _lib.lb_server_clock(self._h)

    def stats(self):
        out = np.zeros(7)
        _lib.lb_server_stats(self._h, _ptr(out))
        keys = ["submitted", "completed", "queued", "running", "device_bytes", "batch_steps", "busy_s"]
        return dict(zip(keys, out.tolist()))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit_decay(t, amp, omega=0.0):
    """lb_fit_decay: decay rate of the amplitude series amp(t) (FP64 least
    squares of ln|amp| on {1, -t}, with omega > 0 also cos/sin(omega t))."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    a = np.ascontiguousarray(amp, dtype=np.float64)
    out = np.zeros(1)
    rc = _lib.lb_fit_decay(_ptr(t), _ptr(a), int(t.size), float(omega), _ptr(out))
    if rc != lb.LB_OK:
        raise lb.LBError(rc, "lb_fit_decay")
    return float(out[0])


def wait_all(server, n, timeout_s=600.0):
    """Poll until n results arrived; returns them."""
    res = []
    t_end = time.time() + timeout_s
    while len(res) < n:
        if time.time() > t_end:
            raise TimeoutError("%d of %d results after %.0f s" % (len(res), n, timeout_s))
        res.extend(server.poll(256, 20000))
    return res


def trace_request(entry, fields):
    """Parameters of the serving-stream request `entry` (see
    workloads.serving_trace): CS D2Q9 in standard lattice units (ds = dt = 1,
    tau = tau_std) or FD D2Q16 (N = 3) on the unit square with the same
    viscosity, tau_FD = (tau_std - 1/2) / (sqrt(3) side), dt = min(CFL 0.5,
    tau_FD), speeds scaled by sqrt(3).  `fields(kind, side, model)` returns
    (rho, ux, uy, probe) and may cache.  Returns submit() keyword arguments."""
    from . import units
    side = entry["side"]
    rho, ux, uy, probe = fields(entry["kind"], side, entry["model"])
    if entry["model"] == "cs":
        return dict(model=lb.LB_CS_D2Q9, Nx=side, Ny=side, tau=entry["tau_std"], dt=1.0, ds=1.0, N=2,
                    rho=rho, ux=ux, uy=uy, nsteps=entry["steps"], probe=probe)
    ds = 1.0 / side
    tau = units.tau_fd_from_std(entry["tau_std"], side)
    dt = units.fd_time_step(tau, ds, 2.3344142183389773, 0.5)
    return dict(model=lb.LB_FD_D2Q16, Nx=side, Ny=side, tau=tau, dt=dt, ds=ds, N=3,
                rho=rho, ux=ux, uy=uy, nsteps=entry["steps"], probe=probe)


def field_cache(u0=0.01):
    """fields(kind, side, model) for trace_request, cached per argument."""
    from . import units, workloads
    cache = {}

    def fields(kind, side, model):
        key = (kind, side, model)
        if key not in cache:
            u = u0 if model == "cs" else units.velocity_fd_from_std(u0)
            cs2 = 1.0 / 3.0 if model == "cs" else 1.0
            if kind == "tgv":
                rho, ux, uy, _ = workloads.taylor_green(side, side, u, cs2)
                probe = workloads.separable_pattern("tgv", side, side)
            else:
                rho, ux, uy, _ = workloads.shear_wave(side, side, u, "y")
                probe = workloads.separable_pattern("shear_y", side, side)
            cache[key] = (rho, ux, uy, probe)
        return cache[key]
    return fields
