"""Stochastic FP16 rounding of the stored state, checked statistically.

On a uniform state every node computes the same FP32 value for a population
(collision-streaming: one rounding per step), so the stored values are the
two FP16 neighbours of that value, and their mean over the nodes equals it to
within the sampling noise (half a step / sqrt(nodes)).  Round-to-nearest
would put every node on the nearer neighbour (a mean off by up to half a
step), and a biased rounding would move the mean by its bias.  The reference
value is the FP64 oracle's step from the same stored initial state; the FP32
arithmetic of the kernel differs from it by a few FP32 ulps of the largest
stored value (`slack`).  For the finite-difference stage kernel the three
Runge-Kutta stages round in turn, so the final values spread over a few
steps around the reference, and the mean test still holds (the stage
combination is affine in the rounded values, the equilibrium smooth in
them).  Cases cover the FP16 normal range and the subnormal range
(|g| < 2^-14, where the FP16 grid is uniform), and the vector and scalar row
forms of the collision-streaming kernel.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import ORACLE_MODEL
from paper_1904_02471_amd import lb

pytestmark = pytest.mark.gpu

SUB = 2.0 ** -14  # smallest normal FP16


def fp16_step(x):
    """Spacing of the FP16 grid at |x|."""
    h = np.abs(np.float16(x))
    return float(np.nextafter(h, np.float16(np.inf))) - float(h) if float(h) >= SUB else 2.0 ** -24


CASES = [
    # model, Nx, Ny, (ux, uy), tau, dt, ds, N
    ("cs vector, normal range", lb.LB_CS_D2Q9, 1024, 1024, (0.0123, -0.0071), 0.6, 1.0, 1.0, 2),
    ("cs vector, pop 0 subnormal", lb.LB_CS_D2Q9, 1024, 1024, (0.0031, 0.0017), 0.6, 1.0, 1.0, 2),
    ("cs scalar rows", lb.LB_CS_D2Q9, 1023, 1024, (0.0123, -0.0071), 0.6, 1.0, 1.0, 2),
    ("fd d2q16", lb.LB_FD_D2Q16, 1024, 1024, (0.0213, -0.0123), 1e-4, 1e-4, 1.0 / 1024, 3),
]


@pytest.mark.parametrize("name,model,Nx,Ny,u,tau,dt,ds,N", CASES, ids=[c[0] for c in CASES])
def test_fp16_rounding_is_unbiased(name, model, Nx, Ny, u, tau, dt, ds, N):
    print("case: fp16 rounding", name, flush=True)
    rho = np.full((Ny, Nx), 1.0 + 3.3e-4)
    # the library's reference density: the mean initial density, summed in
    # node order (repeated additions of one value round systematically, so
    # only the same order reproduces it)
    rho0 = float(np.cumsum(rho.ravel())[-1]) / rho.size
    g = lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=lb.LB_FP16_SHIFTED)
    g.init(rho, np.full((Ny, Nx), u[0]), np.full((Ny, Nx), u[1]))
    f0 = g.get_state()
    g.step(1)
    f1 = g.get_state()
    w = g.w
    K = g.K
    # the FP64 oracle on a small periodic grid from the same (uniform) stored state
    o = oracle.OracleSim(ORACLE_MODEL[model], 8, 8, tau, dt, ds, N)
    o.set_state(np.ascontiguousarray(f0[:, :8, :8]))
    o.step(1)
    ref = o.get_state()[:, 0, 0] - w * rho0
    o.close()

    nodes = Nx * Ny
    gmax = float(np.max(np.abs(ref)))
    slack = 2.0 ** -20 * gmax  # a few FP32 ulps of the largest stored value
    spread = 1 if model == lb.LB_CS_D2Q9 else 4  # FP16 steps the stored values may spread over
    subnormal = 0
    for k in range(K):
        gk = (f1[k] - w[k] * rho0).ravel()
        h = gk.astype(np.float16)
        assert np.all(np.abs(h.astype(np.float64) - gk) <= 1e-12), "stored values are FP16 numbers"
        step = fp16_step(ref[k])
        subnormal += abs(ref[k]) < SUB
        dev = np.abs(gk - ref[k])
        assert dev.max() <= spread * step + slack, (k, dev.max() / step)
        if model == lb.LB_CS_D2Q9:
            # (distinct values counted in float64: numpy's sort of large float16
            # arrays is not reliable here)
            distinct = np.unique(h.astype(np.float64))
            assert len(distinct) <= 2, (k, distinct)
        sigma = 0.5 * spread * step / np.sqrt(nodes)
        bias = float(gk.mean() - ref[k])
        print("pop %2d: g %+.4e step %.2e  mean - ref = %+.2e steps (tol %.2e)"
              % (k, ref[k], step, bias / step, (6 * sigma + slack) / step), flush=True)
        assert abs(bias) <= 6 * sigma + slack, (k, bias / step)
    if "subnormal" in name:
        assert subnormal >= 1
