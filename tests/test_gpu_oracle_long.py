"""FP32 storage against the FP64 oracle over 1000 steps: Taylor-Green
vortices (the 512^2 workload's initial state and relaxation time, on grids
the oracle finishes in seconds) for CS D2Q9, FD D2Q16 (N = 3) and FD D2Q36
(N = 4).  The target is a relative L2 error of at most 1e-5 in the fields
after 1000 steps: u and rho are held to it.  rho - rho0 (about 1e-4 of rho)
is reported beside them and held to what the FP32 rounding of the stored
populations leaves in it (see the test); it does not reach 1e-5."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1904_02471_amd import lb, units, workloads
from tests.gpu_helpers import ORACLE_MODEL, field_errors, rel_l2

pytestmark = pytest.mark.gpu

# host threads of the oracle's row-parallel mode (bitwise its serial run)
THREADS = max(1, min(16, os.cpu_count() or 1))


def tgv_pair(model, n, N, tau_std=0.6, u0=0.01):
    """GPU (FP32) and oracle simulations of the same vortex: CS in standard
    lattice units; FD on the unit box at tau_FD = (tau_std - 1/2)/(sqrt 3 n)
    (the same viscosity), dt = min(CFL 0.5, tau_FD), u scaled to c_s = 1."""
    if model == lb.LB_CS_D2Q9:
        args = (tau_std, 1.0, 1.0, 2)
        rho, ux, uy, _ = workloads.taylor_green(n, n, u0, 1.0 / 3.0)
    else:
        ds = 1.0 / n
        tau = units.tau_fd_from_std(tau_std, n)
        vmax = lb.lb_model_info(model)[0].max()
        args = (tau, units.fd_time_step(tau, ds, vmax, 0.5), ds, N)
        rho, ux, uy, _ = workloads.taylor_green(n, n, units.velocity_fd_from_std(u0), 1.0)
    g = lb.Sim(model, n, n, *args, precision=lb.LB_FP32)
    o = oracle.OracleSim(ORACLE_MODEL[model], n, n, *args)
    o.set_threads(THREADS)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    return g, o


@pytest.mark.parametrize("model,n,N", [(lb.LB_CS_D2Q9, 64, 2), (lb.LB_FD_D2Q16, 64, 3), (lb.LB_FD_D2Q36, 48, 4)],
                         ids=["cs_d2q9_64", "fd_d2q16_64", "fd_d2q36_48"])
def test_tgv_fp32_1000_steps_against_oracle(model, n, N):
    print("case: tgv fp32 vs oracle 1000 steps, model", model, "n", n, flush=True)
    g, o = tgv_pair(model, n, N)
    g.step(1000)
    o.step(1000)
    e_rho, e_u = field_errors(g, o)
    rg, _, _ = g.moments()
    ro, _, _ = o.moments()
    e_full = rel_l2(rg, ro)
    print("1000 steps: rel-L2 u %.2e, rho %.2e, rho - rho0 %.2e (target 1e-5)" % (e_u, e_full, e_rho), flush=True)
    assert e_u <= 1e-5
    assert e_full <= 1e-5
    # rho - rho0 (rms ~7.5e-5) carries the rounding of the stored populations:
    # each rounds by up to 2^-24 of its shifted value (|g| up to ~5e-3, the
    # momentum-carrying part) once per step (CS) or stage (FD); the density
    # sums K of them, and R = 1000 (CS) or 3000 (FD) independent roundings
    # accumulate like a random walk (no credit for the damping of the sound
    # modes that carry them): |d rho| ~ 2^-24 max|g| sqrt(K R)
    f = o.get_state()
    K = f.shape[0]
    vx, vy, w = o.velocities()
    r0 = float(ro.mean())
    gmax = float(np.max(np.abs(f - w[:, None, None] * r0)))
    R = 1000 if model == lb.LB_CS_D2Q9 else 3000
    bound = 2.0 ** -24 * gmax * math.sqrt(K * R) / float(np.sqrt(np.mean((ro - r0) ** 2)))
    print("rho - rho0: rel-L2 %.2e, rounding-noise bound %.2e" % (e_rho, bound), flush=True)
    assert e_rho <= bound
