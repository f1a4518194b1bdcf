"""ctypes binding of liblbm.so, with the names of the C ABI in include/lb.h.

Argument marshalling only: every step of the method runs in the HIP
library.  Importing this module loads liblbm.so and fails loudly when it is
missing; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LB_CS_D2Q9, LB_FD_D2Q9, LB_FD_D2Q16, LB_FD_D2Q25, LB_FD_D2Q36 = 0, 1, 2, 3, 4
LB_FP32, LB_FP16_SHIFTED, LB_FP64, LB_FP16_REF = 0, 1 << 8, 2 << 8, 3 << 8
LB_IMEX = 1 << 10
LB_OK, LB_EINVAL, LB_ECFL, LB_ESTIFF, LB_ENOMEM, LB_EDEVICE, LB_ENAN, LB_EBUSY, LB_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
Q_OF_MODEL = {LB_CS_D2Q9: 3, LB_FD_D2Q9: 3, LB_FD_D2Q16: 4, LB_FD_D2Q25: 5, LB_FD_D2Q36: 6}

# every symbol include/lb.h declares (checked by the CPU test-suite)
EXPORTS = ["lb_create", "lb_destroy", "lb_last_error", "lb_strerror", "lb_model_info", "lb_set_bc_x",
           "lb_set_weno_eps", "lb_init", "lb_step", "lb_moments", "lb_set_probe", "lb_reduce", "lb_reduce_field",
           "lb_reduce_field_noalloc",
           "lb_run_sampled",
           "lb_step_sampled", "lb_series_reserve", "lb_series_read",
           "lb_get_state", "lb_set_state", "lb_steps_done", "lb_set_graph_steps", "lb_set_rounding_seed", "lb_autotune", "lb_set_tuning",
           "lb_set_fd_fused", "lb_get_fd_fused", "lb_tuning_cache_clear", "lb_tuning_cache_size",
           "lb_set_cs_nontemporal", "lb_get_cs_nontemporal",
           "lb_get_tuning", "lb_set_stream", "lb_synchronize",
           "lb_device_bytes",
           "lb_server_create", "lb_server_submit", "lb_server_poll", "lb_server_release", "lb_server_clock",
           "lb_server_stats", "lb_server_destroy", "lb_server_configure", "lb_server_set_node_limit", "lb_server_set_policy", "lb_fit_decay"]

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class LBError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (%s); run paper_1904_02471_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "lb_create": (_vp, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int]),
        "lb_destroy": (None, [_vp]),
        "lb_last_error": (ctypes.c_int, []),
        "lb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "lb_model_info": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]),
        "lb_set_bc_x": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
        "lb_set_weno_eps": (ctypes.c_int, [_vp, ctypes.c_double]),
        "lb_init": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
        "lb_step": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
        "lb_set_probe": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
        "lb_reduce": (ctypes.c_int, [_vp, _dp]),
        "lb_reduce_field": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
        "lb_reduce_field_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "lb_run_sampled": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp]),
        "lb_step_sampled": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
        "lb_series_reserve": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_series_read": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
        "lb_get_state": (ctypes.c_int, [_vp, _dp]),
        "lb_set_state": (ctypes.c_int, [_vp, _dp]),
        "lb_steps_done": (ctypes.c_longlong, [_vp]),
        "lb_set_graph_steps": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_set_rounding_seed": (ctypes.c_int, [_vp, ctypes.c_uint]),
        "lb_autotune": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_tuning_cache_clear": (ctypes.c_int, []),
        "lb_set_cs_nontemporal": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_get_cs_nontemporal": (ctypes.c_int, [_vp]),
        "lb_tuning_cache_size": (ctypes.c_int, []),
        "lb_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "lb_set_fd_fused": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lb_get_fd_fused": (ctypes.c_int, [_vp]),
        "lb_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
        "lb_set_stream": (ctypes.c_int, [_vp, _vp]),
        "lb_synchronize": (ctypes.c_int, [_vp]),
        "lb_device_bytes": (ctypes.c_size_t, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, shape):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape), dtype=np.float64)


def _check(rc, what):
    if rc != LB_OK:
        raise LBError(rc, what)
    return rc


def tuning_cache_clear():
    """Empty the library's autotuning cache (lb_tuning_cache_clear)."""
    _check(_lib.lb_tuning_cache_clear(), "lb_tuning_cache_clear")


def tuning_cache_size():
    """Number of keys in the library's autotuning cache."""
    return int(_lib.lb_tuning_cache_size())


def strerror(code):
    return _lib.lb_strerror(int(code)).decode()


def lb_last_error():
    return _lib.lb_last_error()


def lb_model_info(model, ds=1.0, dt=1.0):
    """(vx, vy, w, cs) of a model."""
    vx, vy, w, cs = np.zeros(64), np.zeros(64), np.zeros(64), np.zeros(1)
    K = _lib.lb_model_info(int(model), float(ds), float(dt), _ptr(vx), _ptr(vy), _ptr(w), _ptr(cs))
    if K < 0:
        raise LBError(K, "lb_model_info")
    return vx[:K].copy(), vy[:K].copy(), w[:K].copy(), float(cs[0])


class Sim:
    """Handle of one simulation: the lb_* calls taking an lb_sim* are its
    methods (same names without the prefix)."""

    def __init__(self, model, Nx, Ny, tau, dt, ds, N=2, precision=LB_FP32, imex=False):
        self.model, self.Nx, self.Ny, self.N = int(model), int(Nx), int(Ny), int(N)
        self.tau, self.dt, self.ds, self.precision = float(tau), float(dt), float(ds), int(precision)
        self.imex = bool(imex)
        flags = self.model | self.precision | (LB_IMEX if self.imex else 0)
        h = _lib.lb_create(flags, self.Nx, self.Ny, self.tau, self.dt, self.ds, self.N)
        if not h:
            raise LBError(_lib.lb_last_error(), "lb_create")
        self._h = h
        q = Q_OF_MODEL[self.model]
        self.K = q * q
        self.vx, self.vy, self.w, self.cs = lb_model_info(self.model, ds, dt)

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_bc_x(self, rho_left, rho_right):
        _check(_lib.lb_set_bc_x(self._h, float(rho_left), float(rho_right)), "lb_set_bc_x")

    def set_weno_eps(self, eps):
        _check(_lib.lb_set_weno_eps(self._h, float(eps)), "lb_set_weno_eps")

    def init(self, rho, ux, uy):
        shp = (self.Ny, self.Nx)
        r, x, y = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        _check(_lib.lb_init(self._h, _ptr(r), _ptr(x), _ptr(y)), "lb_init")

    def step(self, n=1):
        _check(_lib.lb_step(self._h, int(n)), "lb_step")

    def moments(self):
        shp = (self.Ny, self.Nx)
        r, x, y = np.empty(shp), np.empty(shp), np.empty(shp)
        _check(_lib.lb_moments(self._h, _ptr(r), _ptr(x), _ptr(y)), "lb_moments")
        return r, x, y

    def set_probe(self, ax=None, ay=None, bx=None, by=None):
        if ax is None:
            _check(_lib.lb_set_probe(self._h, None, None, None, None), "lb_set_probe")
            return
        a = [_f64(v, (n,)) for v, n in ((ax, self.Nx), (ay, self.Ny), (bx, self.Nx), (by, self.Ny))]
        _check(_lib.lb_set_probe(self._h, *[_ptr(v) for v in a]), "lb_set_probe")

    def reduce(self):
        out = np.empty(5)
        _check(_lib.lb_reduce(self._h, _ptr(out)), "lb_reduce")
        return out

    def reduce_field(self, phi_x=None, phi_y=None):
        """[M, Px, Py, E, A] with A the projection of u on the pattern
        (phi_x, phi_y), two [Ny][Nx] fields (None: A = 0)."""
        out = np.empty(5)
        if phi_x is None and phi_y is None:
            _check(_lib.lb_reduce_field(self._h, None, None, _ptr(out)), "lb_reduce_field")
            return out
        shp = (self.Ny, self.Nx)
        px, py = _f64(phi_x, shp), _f64(phi_y, shp)
        _check(_lib.lb_reduce_field(self._h, _ptr(px), _ptr(py), _ptr(out)), "lb_reduce_field")
        return out

    def reduce_field_noalloc(self, d_phi_x, d_phi_y, d_out):
        """lb_reduce_field_noalloc: device pointers (integers, 0 / None for no
        pattern) of the two [Ny][Nx] FP64 pattern fields and of the 5-double
        output; enqueued on the handle's stream, nothing allocated."""
        _check(_lib.lb_reduce_field_noalloc(self._h, ctypes.c_void_p(int(d_phi_x or 0)),
                                            ctypes.c_void_p(int(d_phi_y or 0)), ctypes.c_void_p(int(d_out or 0))),
               "lb_reduce_field_noalloc")

    def run_sampled(self, nsteps, every):
        n = int(nsteps) // int(every) + 1 if int(every) > 0 and int(nsteps) >= 0 else 1
        out = np.empty((n, 5))
        _check(_lib.lb_run_sampled(self._h, int(nsteps), int(every), _ptr(out)), "lb_run_sampled")
        return out

    def step_sampled(self, nsteps, every):
        _check(_lib.lb_step_sampled(self._h, int(nsteps), int(every)), "lb_step_sampled")

    def series_reserve(self, capacity):
        _check(_lib.lb_series_reserve(self._h, int(capacity)), "lb_series_reserve")

    def series_read(self, max_rows=1 << 16):
        out = np.empty((int(max_rows), 6))
        n = _lib.lb_series_read(self._h, _ptr(out), int(max_rows))
        if n < 0:
            raise LBError(n, "lb_series_read")
        return out[:n].copy()

    def get_state(self):
        f = np.empty((self.K, self.Ny, self.Nx))
        _check(_lib.lb_get_state(self._h, _ptr(f)), "lb_get_state")
        return f

    def set_state(self, f):
        f = _f64(f, (self.K, self.Ny, self.Nx))
        _check(_lib.lb_set_state(self._h, _ptr(f)), "lb_set_state")

    def steps_done(self):
        return _lib.lb_steps_done(self._h)

    def set_graph_steps(self, steps):
        """Steps per replayed HIP graph for runs of plain steps (-1: default, 0: off)."""
        _check(_lib.lb_set_graph_steps(self._h, int(steps)), "lb_set_graph_steps")

    def set_rounding_seed(self, seed):
        """FP16 storage: the random-bit stream of the stochastic rounding (0 by default)."""
        _check(_lib.lb_set_rounding_seed(self._h, int(seed)), "lb_set_rounding_seed")

    def autotune(self, reps=20):
        """Time the plain-step launch shapes on this simulation and keep the fastest."""
        _check(_lib.lb_autotune(self._h, int(reps)), "lb_autotune")
        return self.tuning()

    def set_tuning(self, cs_threads, fd_rows, fd_rows_rest=None):
        """fd_rows: tile rows of the first FD stage, fd_rows_rest: of the
        later stages (default: the same)."""
        rest = fd_rows if fd_rows_rest is None else fd_rows_rest
        _check(_lib.lb_set_tuning(self._h, int(cs_threads), int(fd_rows), int(rest)), "lb_set_tuning")

    def set_fd_fused(self, rows_per_segment):
        """FD plain steps by the temporally blocked kernel with y-segments of
        this many rows (0: the three stage launches)."""
        _check(_lib.lb_set_fd_fused(self._h, int(rows_per_segment)), "lb_set_fd_fused")

    def fd_fused(self):
        return _lib.lb_get_fd_fused(self._h)

    def set_cs_nontemporal(self, on):
        """CS plain steps: non-temporal (True) or plain (False) stores."""
        _check(_lib.lb_set_cs_nontemporal(self._h, 1 if on else 0), "lb_set_cs_nontemporal")

    def cs_nontemporal(self):
        return bool(_lib.lb_get_cs_nontemporal(self._h))

    def tuning(self):
        """(cs_threads, fd_rows, fd_rows_rest) of the plain steps."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.lb_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "lb_get_tuning")
        return a.value, b.value, c.value

    def set_stream(self, stream_handle):
        """stream_handle: an integer hipStream_t (e.g. torch.cuda.Stream().cuda_stream) or 0/None."""
        _check(_lib.lb_set_stream(self._h, ctypes.c_void_p(int(stream_handle or 0))), "lb_set_stream")

    def synchronize(self):
        _check(_lib.lb_synchronize(self._h), "lb_synchronize")

    def device_bytes(self):
        return _lib.lb_device_bytes(self._h)
