"""Implicit-explicit FD stepping (LB_IMEX) on the GPU: element-wise parity
with the oracle's IMEX-SSP2(2,2,2) steps (also at dt > tau), graph replay,
and the stiff shock tube (dt = 14 tau) against the exact solution."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1904_02471_amd import lb, workloads
from tests.gpu_helpers import ORACLE_MODEL, PREC_NAME, assert_state_close, rel_l2, tolerance

pytestmark = pytest.mark.gpu


def imex_pair(model, Nx, Ny, tau, dt, N, prec, bc=None):
    ds = 1.0 / Nx
    g = lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=prec, imex=True)
    o = oracle.OracleSim(ORACLE_MODEL[model], Nx, Ny, tau, dt, ds, N)
    o.set_time_scheme(1)
    if bc is not None:
        g.set_bc_x(*bc)
        o.set_bc_x(*bc)
    return g, o


@pytest.mark.parametrize("prec", [lb.LB_FP64, lb.LB_FP32, lb.LB_FP16_SHIFTED], ids=lambda p: PREC_NAME[p])
@pytest.mark.parametrize("model,N,Nx,Ny,dt_over_tau", [
    (lb.LB_FD_D2Q16, 3, 70, 37, 2.0),
    (lb.LB_FD_D2Q36, 4, 33, 20, 0.5),
    (lb.LB_FD_D2Q9, 2, 64, 33, 20.0),
])
def test_imex_matches_oracle(model, N, Nx, Ny, dt_over_tau, prec):
    print("case: imex parity", model, Nx, Ny, dt_over_tau, PREC_NAME[prec], flush=True)
    vmax = lb.lb_model_info(model)[0].max()
    dt = 0.4 / (Nx * vmax)
    g, o = imex_pair(model, Nx, Ny, dt / dt_over_tau, dt, N, prec)
    f0 = workloads.random_distribution(g.K, Nx, Ny, 41 + Nx, g.w, spread=0.2)
    g.set_state(f0)
    o.set_state(f0)
    done = 0
    for n in (1, 4, 9):
        g.step(n - done)
        o.step(n - done)
        done = n
        fo = o.get_state()
        # four stored stages per step instead of three (twice the per-step
        # bound of the Runge-Kutta path).  In FP16 the pointwise stages also
        # combine stored values with weights up to 3 (h = y + 3 (g - f1),
        # b = 2 f1 + h - g - f2), and the stencil stage evaluates the
        # relaxation of the stored f1 explicitly, which multiplies its
        # rounding by dt / tau: (12 + dt / tau) FP16 roundings of max|g|
        rho0 = fo.sum(0).mean()
        tol = 2 * tolerance(prec, n, fo, g.w, rho0)
        if prec == lb.LB_FP16_SHIFTED:
            gmax = float(np.max(np.abs(fo - g.w[:, None, None] * rho0)))
            tol = 2 * tolerance(lb.LB_FP32, n, fo, g.w, rho0) + (12 + dt_over_tau) * 2.0 ** -11 * (n + 1) * gmax
        assert_state_close(g.get_state(), fo, tol, "imex %s after %d steps" % (PREC_NAME[prec], n))


def test_imex_fixed_ends_and_graphs():
    print("case: imex fixed ends, graphs", flush=True)
    Nx, Ny, tau = 48, 10, 1e-4
    dt = 0.4 / (Nx * math.sqrt(3))
    g, o = imex_pair(lb.LB_FD_D2Q9, Nx, Ny, tau, dt, 2, lb.LB_FP64, bc=(1.2, 1.0))
    rho, ux, uy = workloads.shock_tube(Nx, Ny, 1.2, 1.0)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    g.step(11)   # two 4-step graphs and three single steps
    o.step(11)
    fo = o.get_state()
    assert_state_close(g.get_state(), fo, 2 * tolerance(lb.LB_FP64, 11, fo, g.w, 1.1), "imex fixed ends")
    e = lb.Sim(lb.LB_FD_D2Q9, Nx, Ny, tau, dt, 1.0 / Nx, 2, precision=lb.LB_FP64, imex=True)
    e.set_bc_x(1.2, 1.0)
    e.set_graph_steps(0)
    e.init(rho, ux, uy)
    e.step(11)
    assert np.array_equal(e.get_state(), g.get_state())


def test_stiff_shock_tube_2048():
    """2048 x 4 periodic, rho 1.1 / 0.9 (the setup of Section 4.1) at
    tau_FD = 1e-5 with dt at CFL 0.5 (14 tau), which the explicit collision
    cannot run: FP64 and FP32 reach the exact plateau, and agree."""
    print("case: stiff shock tube", flush=True)
    n, rl, rr, tau = 2048, 1.1, 0.9, 1e-5
    dt = 0.5 / (n * math.sqrt(3))
    assert dt > 10 * tau
    with pytest.raises(lb.LBError):
        lb.Sim(lb.LB_FD_D2Q9, n, 4, tau, dt, 1.0 / n, 2)     # explicit: LB_ESTIFF
    steps = int(round(0.1128 / dt))
    rho0, ux0, uy0 = workloads.shock_tube(n, 4, rl, rr)
    prof = {}
    for prec in (lb.LB_FP64, lb.LB_FP32):
        s = lb.Sim(lb.LB_FD_D2Q9, n, 4, tau, dt, 1.0 / n, 2, precision=prec, imex=True)
        s.init(rho0, ux0, uy0)
        s.step(steps)
        r, u, _ = s.moments()
        prof[prec] = (r[0], u[0])
    sol = exact.riemann_solution(rl, rr, 1.0)
    x = (np.arange(n) + 0.5) / n
    xi = (x - 0.5) / (steps * dt)
    lo, hi = sol["xi_c"], sol["xi_s"]
    mid = (xi > lo + 0.25 * (hi - lo)) & (xi < hi - 0.25 * (hi - lo))
    r, u = prof[lb.LB_FP64]
    print("plateau rho %.5f u %.5f (exact %.5f %.5f)" % (r[mid].mean(), u[mid].mean(), sol["rho_c"], sol["u_c"]),
          flush=True)
    assert np.max(np.abs(r[mid] - sol["rho_c"])) < 2e-3
    assert np.max(np.abs(u[mid] - sol["u_c"])) < 4e-3
    e = rel_l2(prof[lb.LB_FP32][0] - 1.0, r - 1.0)
    print("fp32 vs fp64 density rel-L2 %.2e" % e, flush=True)
    assert e < 1e-4
