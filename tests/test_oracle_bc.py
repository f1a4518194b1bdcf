"""Pins of the oracle's boundary handling and of its nonlinear dynamics on
the shock tube (Section 4.1) and the Taylor-Green vortex (Section 4.3)."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1904_02471_amd import workloads

E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])


def test_cs_fixed_ends_one_step():
    # with fixed ends, populations entering at x = 0 (E, NE, SE) and at
    # x = Nx-1 (W, NW, SW) come from the end equilibria; all others are as
    # in the periodic step.
    rng = np.random.default_rng(8)
    Nx, Ny = 7, 6
    f = workloads.random_distribution(9, Nx, Ny, 8, oracle.velocity_set(0)[2])
    per = oracle.OracleSim(oracle.CS_D2Q9, Nx, Ny, 0.7, 1.0, 1.0, 2)
    fix = oracle.OracleSim(oracle.CS_D2Q9, Nx, Ny, 0.7, 1.0, 1.0, 2)
    fix.set_bc_x(1.3, 0.8)
    per.set_state(f)
    fix.set_state(f)
    per.step(1)
    fix.step(1)
    a, b = per.get_state(), fix.get_state()
    fl, fr = fix.equilibrium(1.3, 0, 0), fix.equilibrium(0.8, 0, 0)
    for k in range(9):
        inner = np.ones((Ny, Nx), bool)
        if E[k, 0] == 1:
            inner[:, 0] = False
            assert np.all(b[k][:, 0] == fl[k])
        if E[k, 0] == -1:
            inner[:, -1] = False
            assert np.all(b[k][:, -1] == fr[k])
        assert np.array_equal(a[k][inner], b[k][inner])


@pytest.mark.parametrize("model,N", [(oracle.CS_D2Q9, 2), (oracle.FD_D2Q16, 3)])
def test_matching_end_state_is_steady(model, N):
    Nx, Ny = 12, 3
    if model == oracle.CS_D2Q9:
        sim = oracle.OracleSim(model, Nx, Ny, 0.7, 1.0, 1.0, N)
    else:
        sim = oracle.OracleSim(model, Nx, Ny, 1e-3, 1e-3, 1.0 / Nx, N)
    sim.set_bc_x(1.2, 1.2)
    sim.init(np.full((Ny, Nx), 1.2), np.zeros((Ny, Nx)), np.zeros((Ny, Nx)))
    f0 = sim.get_state()
    sim.step(10)
    np.testing.assert_allclose(sim.get_state(), f0, rtol=1e-13)


def plateau_check(rho, u, x, t, rl, rr, cs, tol):
    s = exact.riemann_solution(rl, rr, cs)
    x0 = 0.5
    xi = (x - x0) / t
    mid = (xi > s["xi_c"] + 0.25 * (s["xi_s"] - s["xi_c"])) & (xi < s["xi_s"] - 0.25 * (s["xi_s"] - s["xi_c"]))
    assert mid.sum() >= 5
    assert np.max(np.abs(rho[mid] / s["rho_c"] - 1)) < tol
    assert np.max(np.abs(u[mid] - s["u_c"])) < tol * cs
    # shock position: where rho crosses the midpoint between plateau and right state
    half = 0.5 * (s["rho_c"] + rr)
    right = x > x0
    idx = np.where(right & (rho < half))[0][0]
    x_s = x[idx - 1] + (rho[idx - 1] - half) / (rho[idx - 1] - rho[idx]) * (x[idx] - x[idx - 1])
    return x_s - (x0 + s["xi_s"] * t)


@pytest.mark.parametrize("fixed", [False, True])
def test_shock_tube_fd_against_exact(fixed):
    """FD D2Q9 (N = 2), N_x = 256, rho 1.1 / 0.9, tau_FD = 1e-4, dt at CFL
    0.5, up to t = 0.1128 (Section 4.1)."""
    Nx, rl, rr = 256, 1.1, 0.9
    ds = 1.0 / Nx
    tau = 1e-4
    dt = min(0.5 * ds / math.sqrt(3), tau)
    steps = int(round(0.1128 / dt))
    sim = oracle.OracleSim(oracle.FD_D2Q9, Nx, 1, tau, dt, ds, 2)
    if fixed:
        sim.set_bc_x(rl, rr)
    rho0, ux0, uy0 = workloads.shock_tube(Nx, 1, rl, rr)
    sim.init(rho0, ux0, uy0)
    sim.step(steps)
    rho, ux, _ = sim.moments()
    x = np.arange(Nx) * ds + 0.5 * ds        # node i sits at (i + 1/2) ds from the step at x0 = 1/2
    off = plateau_check(rho[0], ux[0], x, steps * dt, rl, rr, 1.0, 2e-3)
    assert abs(off) < 3 * ds


def test_shock_tube_cs_against_exact():
    """CS D2Q9 in the paper's units (ds = 1, dt = 1/sqrt 3, c_s = 1), N = 256,
    tau_LU = N tau_FD + sqrt(3)/6 with tau_FD = 1e-3."""
    Nx, rl, rr = 256, 1.1, 0.9
    tau = exact.tau_lu_from_fd(1e-3, Nx)
    dt = 1 / math.sqrt(3)
    steps = int(round(0.1128 * Nx / dt))
    sim = oracle.OracleSim(oracle.CS_D2Q9, Nx, 1, tau, dt, 1.0, 2)
    rho0, ux0, uy0 = workloads.shock_tube(Nx, 1, rl, rr)
    sim.init(rho0, ux0, uy0)
    sim.step(steps)
    rho, ux, _ = sim.moments()
    x = (np.arange(Nx) + 0.5) / Nx
    off = plateau_check(rho[0], ux[0], x, steps * dt / Nx, rl, rr, 1.0, 3e-3)
    assert abs(off) < 6.0 / Nx


def test_taylor_green_cs_decay():
    """CS D2Q9 32 x 32, tau = 0.6 (ds = dt = 1): amplitude decays as
    exp(-2 k^2 nu t) with nu = (tau - 1/2)/3 up to the lattice error."""
    N, tau, U = 32, 0.6, 0.01
    sim = oracle.OracleSim(oracle.CS_D2Q9, N, N, tau, 1.0, 1.0, 2)
    rho, ux, uy, (px, py) = workloads.taylor_green(N, N, U, 1.0 / 3.0)
    sim.init(rho, ux, uy)
    t, a = [], []
    for n in range(0, 601, 20):
        if n:
            sim.step(20)
        if n >= 40:
            t.append(float(n))
            a.append(sim.reduce(px, py)[4])
    k = 2 * math.pi / N
    nu = exact.apparent_viscosity(t, a, k, "tgv")
    assert nu == pytest.approx((tau - 0.5) / 3, rel=5e-3)
