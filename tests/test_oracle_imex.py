"""Pins of the oracle's implicit-explicit time stepping (FD models): the
properties that fix a second-order, L-stable IMEX Runge-Kutta scheme for the
BGK relaxation, conservation, second-order convergence with advection, and
stability in the stiff regime where the explicit scheme fails."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1904_02471_amd import workloads


def fd_sim(model, Nx, Ny, tau, dt, N, scheme):
    s = oracle.OracleSim(model, Nx, Ny, tau, dt, 1.0 / Nx, N)
    s.set_time_scheme(scheme)
    return s


def relaxation_factor(dt_over_tau):
    """Decay factor of a uniform non-equilibrium perturbation over one step
    (no advection for a uniform state; f_eq fixed by the conserved moments)."""
    s = fd_sim(oracle.FD_D2Q9, 4, 3, 1.0, dt_over_tau, 2, 1)
    vx, vy, w = s.velocities()
    feq = s.equilibrium(1.02, 0.03, -0.01)
    delta = 1e-3 * w * (vx * vx - 1.0)  # zero mass and momentum
    f = np.broadcast_to((feq + delta)[:, None, None], (9, 3, 4)).copy()
    s.set_state(f)
    s.step(1)
    out = s.get_state()[:, 1, 2]
    return (out - feq) @ delta / (delta @ delta)


def test_relaxation_is_second_order_and_l_stable():
    # second order: the one-step error against exp(-dt/tau) scales as (dt/tau)^3
    e = [abs(relaxation_factor(z) - math.exp(-z)) for z in (0.04, 0.02, 0.01)]
    assert e[0] / e[1] == pytest.approx(8.0, rel=0.05)
    assert e[1] / e[2] == pytest.approx(8.0, rel=0.05)
    # L-stable: a step much longer than tau removes the non-equilibrium part
    for z in (1e3, 1e6):
        assert abs(relaxation_factor(z)) < 10.0 / z
    # and never amplifies it
    for z in (0.5, 2.0, 10.0, 100.0):
        assert abs(relaxation_factor(z)) < 1.0


def test_conservation_random_state():
    s = fd_sim(oracle.FD_D2Q16, 12, 10, 2e-3, 4e-3, 3, 1)   # dt = 2 tau
    vx, vy, w = s.velocities()
    f0 = workloads.random_distribution(16, 12, 10, 77, w, spread=0.3)
    s.set_state(f0)
    s.step(5)
    f = s.get_state()
    for wt in (np.ones(16), vx, vy):
        m0 = np.tensordot(wt, f0, 1).sum()
        m1 = np.tensordot(wt, f, 1).sum()
        assert abs(m1 - m0) <= 1e-13 * max(1.0, abs(m0))


def test_second_order_in_time_with_advection():
    """Shear wave, FD D2Q9 on 32 nodes, tau = 2e-3: the state at t = 0.08 from
    IMEX steps dt, dt/2, dt/4 converges at second order to the RK-3 limit."""
    n, tau, t_end = 32, 2e-3, 0.08
    rho, ux, uy, _ = workloads.shear_wave(n, 1, 0.01, "x")

    def run(scheme, dt):
        s = fd_sim(oracle.FD_D2Q9, n, 1, tau, dt, 2, scheme)
        s.init(rho, ux, uy)
        s.step(int(round(t_end / dt)))
        return s.get_state()

    ref = run(0, t_end / 1280)
    errs = [np.abs(run(1, dt) - ref).max() for dt in (t_end / 40, t_end / 80, t_end / 160)]
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.2)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.2)


def test_stiff_shock_tube():
    """dt = 10 tau: the explicit collision blows up, the IMEX step stays
    bounded and gives the inviscid plateau of the isothermal Riemann problem."""
    n, rl, rr = 256, 1.1, 0.9
    tau = 1e-5
    dt = 0.5 / (n * math.sqrt(3.0))  # CFL 0.5 for the D2Q9 velocities +-sqrt(3)
    assert dt > 10 * tau
    steps = int(round(0.1 / dt))
    rho0, ux0, uy0 = workloads.shock_tube(n, 1, rl, rr)
    rk = fd_sim(oracle.FD_D2Q9, n, 1, tau, dt, 2, 0)
    rk.init(rho0, ux0, uy0)
    rk.step(3)
    with np.errstate(all="ignore"):
        assert not np.all(np.abs(rk.get_state()) < 10.0)
    s = fd_sim(oracle.FD_D2Q9, n, 1, tau, dt, 2, 1)
    s.init(rho0, ux0, uy0)
    s.step(steps)
    r, u, _ = s.moments()
    assert np.all(np.isfinite(r)) and r.min() > 0.8 and r.max() < 1.2
    sol = exact.riemann_solution(rl, rr, 1.0)
    x = (np.arange(n) + 0.5) / n
    xi = (x - 0.5) / (steps * dt)
    lo, hi = sol["xi_c"], sol["xi_s"]
    mid = (xi > lo + 0.25 * (hi - lo)) & (xi < hi - 0.25 * (hi - lo))
    assert np.max(np.abs(r[0, mid] - sol["rho_c"])) < 5e-3
    assert np.max(np.abs(u[0, mid] - sol["u_c"])) < 1e-2
