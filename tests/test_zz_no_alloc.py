"""lb_reduce_field_noalloc (the entry point for callers that cannot allocate
device memory) against lb_reduce_field, through the C ABI: bitwise the same
diagnostics on two calls in a row, the second on a smaller grid, with and
without a pattern."""
import ctypes

import numpy as np
import pytest

from paper_1904_02471_amd import lb, workloads

pytestmark = pytest.mark.gpu


class HipRuntime:
    """The test's own device buffers, from the HIP runtime that liblbm.so
    runs on (already loaded with the library: the same SONAME resolves to it)."""

    def __init__(self):
        lib = ctypes.CDLL("libamdhip64.so.7")
        lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        lib.hipMalloc.restype = ctypes.c_int
        lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        lib.hipMemcpy.restype = ctypes.c_int
        lib.hipFree.argtypes = [ctypes.c_void_p]
        lib.hipFree.restype = ctypes.c_int
        self.lib = lib

    def upload(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        p = ctypes.c_void_p()
        assert self.lib.hipMalloc(ctypes.byref(p), a.nbytes) == 0
        assert self.lib.hipMemcpy(p, a.ctypes.data_as(ctypes.c_void_p), a.nbytes, 1) == 0  # host to device
        return p.value

    def download(self, ptr, n):
        out = np.empty(n)
        assert self.lib.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ptr), out.nbytes, 2) == 0
        return out

    def free(self, ptr):
        if ptr:
            assert self.lib.hipFree(ctypes.c_void_p(ptr)) == 0


def noalloc_reduce(hip, sim, px, py):
    d_out = hip.upload(np.full(5, np.nan))
    d_x = hip.upload(px) if px is not None else None
    d_y = hip.upload(py) if py is not None else None
    try:
        sim.reduce_field_noalloc(d_x, d_y, d_out)   # synchronous copies above: the inputs are in place
        sim.synchronize()
        return hip.download(d_out, 5)
    finally:
        for p in (d_out, d_x, d_y):
            hip.free(p)


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_allocating_entry_point(order):
    cases = [(lb.LB_CS_D2Q9, 512, 512), (lb.LB_FD_D2Q16, 70, 45)]  # 1024 partial blocks, then 13
    rng = np.random.default_rng(1906)
    hip = HipRuntime()
    for model, Nx, Ny in cases:
        print("case: noalloc reduce model", model, Nx, Ny, flush=True)
        if model == lb.LB_CS_D2Q9:
            sim = lb.Sim(model, Nx, Ny, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP32)
        else:
            ds = 1.0 / Nx
            dt = 0.5 * ds / 2.3344142183389773
            sim = lb.Sim(model, Nx, Ny, 2 * dt, dt, ds, 3, precision=lb.LB_FP32)
        rho, ux, uy = workloads.random_state(Nx, Ny, 5 + Nx, sim.cs, u_max=0.05)
        sim.init(rho, ux, uy)
        sim.step(2)
        px, py = rng.standard_normal((Ny, Nx)), rng.standard_normal((Ny, Nx))
        want = sim.reduce_field(px, py)
        got = noalloc_reduce(hip, sim, px, py)
        print("noalloc", got, "allocating", want, flush=True)
        assert np.array_equal(got, want)
        want0 = sim.reduce_field()
        got0 = noalloc_reduce(hip, sim, None, None)
        assert np.array_equal(got0, want0) and got0[4] == 0.0
        sim.destroy()


def test_noalloc_argument_checks():
    sim = lb.Sim(lb.LB_CS_D2Q9, 8, 8, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP32)
    with pytest.raises(lb.LBError) as e:
        sim.reduce_field_noalloc(0, 0, 0)          # no output
    assert e.value.code == lb.LB_EINVAL
    with pytest.raises(lb.LBError) as e:
        sim.reduce_field_noalloc(0, 0, 4096)       # before init
    assert e.value.code == lb.LB_ESTATE
    sim.destroy()
