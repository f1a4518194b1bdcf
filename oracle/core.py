"""ctypes binding of the FP64 CPU oracle (lb_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never loads this.
"""
import ctypes
import os

import numpy as np

from . import build as _build

CS_D2Q9, FD_D2Q9, FD_D2Q16, FD_D2Q25, FD_D2Q36 = 0, 1, 2, 3, 4

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        _build.build(force=True)
    lib = ctypes.CDLL(path)
    lib.orc_gauss_hermite.argtypes = [ctypes.c_int, _dp, _dp]
    lib.orc_gauss_hermite.restype = ctypes.c_int
    lib.orc_velocity_set.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _ip, _ip]
    lib.orc_velocity_set.restype = ctypes.c_int
    lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int]
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_num_populations.argtypes = [ctypes.c_void_p]
    lib.orc_num_populations.restype = ctypes.c_int
    lib.orc_sound_speed.argtypes = [ctypes.c_void_p]
    lib.orc_sound_speed.restype = ctypes.c_double
    lib.orc_velocities.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_set_weno_eps.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.orc_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_set_time_scheme.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_set_bc_x.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    lib.orc_equilibrium.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_get_state.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_set_state.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_reduce.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_weno5.argtypes = [ctypes.c_double] * 6
    lib.orc_weno5.restype = ctypes.c_double
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)
    return a


def gauss_hermite(Q):
    """Roots (ascending) and normalised weights of the Q-point Gauss-Hermite
    rule for the weight exp(-x^2/2)/sqrt(2 pi) (Section 1)."""
    lib = _load()
    x = np.zeros(Q)
    w = np.zeros(Q)
    if lib.orc_gauss_hermite(Q, _ptr(x), _ptr(w)) != 0:
        raise ValueError("gauss_hermite failed for Q=%d" % Q)
    return x, w


def velocity_set(model, ds=1.0, dt=1.0):
    """(vx, vy, w, cs) of a model; CS D2Q9 in units of ds/dt, FD with c_s=1."""
    lib = _load()
    vx, vy, w = np.zeros(64), np.zeros(64), np.zeros(64)
    cs = np.zeros(1)
    K = lib.orc_velocity_set(model, ds, dt, _ptr(vx), _ptr(vy), _ptr(w), _ptr(cs), None, None)
    if K < 0:
        raise ValueError("bad model %r" % model)
    return vx[:K].copy(), vy[:K].copy(), w[:K].copy(), float(cs[0])


def weno5(a, b, c, d, e, eps=1e-6):
    return _load().orc_weno5(a, b, c, d, e, eps)


class OracleSim:
    """One simulation held by the oracle.  Same call sequence as the GPU
    library: create -> init -> step -> moments / reduce / get_state."""

    def __init__(self, model, Nx, Ny, tau, dt, ds, N=2):
        lib = _load()
        self._lib = lib
        self._h = lib.orc_create(model, Nx, Ny, tau, dt, ds, N)
        if not self._h:
            raise ValueError("oracle rejected parameters model=%r Nx=%r Ny=%r tau=%r dt=%r ds=%r N=%r"
                             % (model, Nx, Ny, tau, dt, ds, N))
        self.model, self.Nx, self.Ny, self.N = model, Nx, Ny, N
        self.tau, self.dt, self.ds = tau, dt, ds
        self.K = lib.orc_num_populations(self._h)
        self.cs = lib.orc_sound_speed(self._h)

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def velocities(self):
        vx, vy, w = np.zeros(self.K), np.zeros(self.K), np.zeros(self.K)
        self._lib.orc_velocities(self._h, _ptr(vx), _ptr(vy), _ptr(w))
        return vx, vy, w

    def set_weno_eps(self, eps):
        self._lib.orc_set_weno_eps(self._h, eps)

    def set_threads(self, threads):
        """Host threads of the row and node loops (1, the default, is the plain
        serial run); the results are bitwise the same for any count."""
        self._lib.orc_set_threads(self._h, int(threads))

    def set_time_scheme(self, scheme):
        """FD only: 0 third-order TVD Runge-Kutta, 1 IMEX-SSP2(2,2,2) (advection
        explicit, BGK relaxation implicit)."""
        self._lib.orc_set_time_scheme(self._h, int(scheme))

    def set_bc_x(self, rho_left, rho_right):
        self._lib.orc_set_bc_x(self._h, rho_left, rho_right)

    def equilibrium(self, rho, ux, uy):
        out = np.zeros(self.K)
        self._lib.orc_equilibrium(self._h, rho, ux, uy, _ptr(out))
        return out

    def init(self, rho, ux, uy):
        shp = (self.Ny, self.Nx)
        r, x, y = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        self._lib.orc_init(self._h, _ptr(r), _ptr(x), _ptr(y))

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    def moments(self):
        shp = (self.Ny, self.Nx)
        r, x, y = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        self._lib.orc_moments(self._h, _ptr(r), _ptr(x), _ptr(y))
        return r, x, y

    def get_state(self):
        f = np.zeros((self.K, self.Ny, self.Nx))
        self._lib.orc_get_state(self._h, _ptr(f))
        return f

    def set_state(self, f):
        f = _f64(f, (self.K, self.Ny, self.Nx))
        self._lib.orc_set_state(self._h, _ptr(f))

    def reduce(self, phi_x=None, phi_y=None):
        out = np.zeros(5)
        if phi_x is None:
            self._lib.orc_reduce(self._h, None, None, _ptr(out))
        else:
            shp = (self.Ny, self.Nx)
            px, py = _f64(phi_x, shp), _f64(phi_y, shp)
            self._lib.orc_reduce(self._h, _ptr(px), _ptr(py), _ptr(out))
        return out
