"""Pins of the oracle's finite-difference step (Section 2: BGK equation
advanced with TVD RK-3 in time and WENO-5 advection; nu_FD = tau_FD T/m)."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact


# ---------------------------------------------------------------- WENO-5 ---

def test_weno_quadratic_exactness():
    # Finite-difference WENO reconstructs h at the interface, where the data
    # are cell averages of h.  For f = x^2 sampled at x_i = i, h = x^2 - 1/12,
    # and every candidate stencil is exact, whatever the nonlinear weights.
    for c0 in [-3.0, 0.0, 2.5]:
        vals = [(c0 + m) ** 2 for m in range(-2, 3)]
        want = (c0 + 0.5) ** 2 - 1.0 / 12.0
        for eps in [1e-6, 1e-40, 1e30]:
            assert oracle.weno5(*vals, eps) == pytest.approx(want, rel=1e-13, abs=1e-13)


def test_weno_linear_limit_is_upwind5():
    # eps much larger than every smoothness indicator gives the linear weights
    # (1/10, 6/10, 3/10): the classic fifth-order upwind-biased flux
    # (2 a - 13 b + 47 c + 27 d - 3 e) / 60.
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b, c, d, e = rng.standard_normal(5)
        want = (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60
        assert oracle.weno5(a, b, c, d, e, 1e30) == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_weno_linear_data_gives_linear_weights():
    # for linear data the three smoothness indicators are all equal
    for eps in [1e-6, 1e-12]:
        vals = [0.3 + 0.1 * m for m in range(-2, 3)]
        want = (2 * vals[0] - 13 * vals[1] + 47 * vals[2] + 27 * vals[3] - 3 * vals[4]) / 60
        assert oracle.weno5(*vals, eps) == pytest.approx(want, rel=1e-14)


def test_weno_essentially_non_oscillatory_at_a_jump():
    # jump between the upwind cell c and d: the reconstruction keeps the
    # upwind-side value (the smooth stencil q0 dominates), no overshoot.
    got = oracle.weno5(1.0, 1.0, 1.0, 0.0, 0.0, 1e-6)
    assert abs(got - 1.0) < 1e-9
    got = oracle.weno5(1.0, 1.0, 0.0, 0.0, 0.0, 1e-6)
    assert abs(got - 0.0) < 1e-9
    # a linear reconstruction would overshoot
    assert (2 - 13 + 47) / 60 > 0.5


def upwind5_symbol(theta, positive):
    """Fourier symbol of F_{i+1/2} - F_{i-1/2} for the linear upwind-5 flux."""
    c = np.array([2, -13, 47, 27, -3]) / 60.0
    if positive:
        offs = np.array([-2, -1, 0, 1, 2])
    else:
        offs = np.array([3, 2, 1, 0, -1])
    cf = np.sum(c * np.exp(1j * offs * theta))
    return cf * (1 - np.exp(-1j * theta))


def test_upwind5_symbol_is_fifth_order():
    # guard of the pin itself: D(theta) = i theta + O(theta^6)
    for positive in (True, False):
        errs = [abs(upwind5_symbol(th, positive) - 1j * th) for th in (0.1, 0.05)]
        order = math.log(errs[0] / errs[1]) / math.log(2)
        assert order == pytest.approx(6.0, abs=0.1)


# ------------------------------------------------------------- full step ---

def linear_fd_matrix(q, ds, dt, tau, vx, vy, w):
    """One RK-3 step linearised at rho = 1, u = 0 for the mode exp(i q.x)
    (x in node units), with the linear upwind-5 flux.  L = -diag(v D)/ds -
    (I - Eq)/tau, and the Shu-Osher RK-3 of a linear system is the cubic
    Taylor polynomial I + hL + (hL)^2/2 + (hL)^3/6."""
    K = len(w)
    xi = np.stack([vx, vy], 1)
    Eq = w[:, None] * (1.0 + xi @ xi.T)
    adv = np.zeros(K, dtype=complex)
    for k in range(K):
        if vx[k] != 0:
            adv[k] += vx[k] * upwind5_symbol(q[0], vx[k] > 0)
        if vy[k] != 0:
            adv[k] += vy[k] * upwind5_symbol(q[1], vy[k] > 0)
    L = -np.diag(adv) / ds - (np.eye(K) - Eq) / tau
    hL = dt * L
    return np.eye(K) + hL + hL @ hL / 2 + hL @ hL @ hL / 6


@pytest.mark.parametrize("model,N", [(oracle.FD_D2Q9, 2), (oracle.FD_D2Q16, 3), (oracle.FD_D2Q25, 2),
                                     (oracle.FD_D2Q36, 4)])
def test_linear_response_one_step(model, N):
    Nx, Ny = 12, 10
    ds, tau = 1.0 / 12, 2e-3
    dt = 0.4 * ds / 3.4 if model == oracle.FD_D2Q36 else 0.5 * ds / 2.4
    dt = min(dt, tau)
    sim = oracle.OracleSim(model, Nx, Ny, tau, dt, ds, N)
    sim.set_weno_eps(1e30)            # linear limit of the reconstruction
    vx, vy, w = sim.velocities()
    K = len(w)
    rng = np.random.default_rng(4 + model)
    X, Y = np.meshgrid(np.arange(Nx), np.arange(Ny))
    for m, n in [(1, 0), (0, 1), (2, 3), (5, 4)]:
        q = 2 * np.pi * np.array([m / Nx, n / Ny])
        a = rng.standard_normal(K) + 1j * rng.standard_normal(K)
        phase = np.exp(1j * (q[0] * X + q[1] * Y))
        pert = np.real(a[:, None, None] * phase)
        eps = 1e-6
        out = []
        for sgn in (1.0, -1.0):
            sim.set_state(w[:, None, None] + sgn * eps * pert)
            sim.step(1)
            out.append(sim.get_state())
        got = (out[0] - out[1]) / (2 * eps)
        a1 = linear_fd_matrix(q, ds, dt, tau, vx, vy, w) @ a
        want = np.real(a1[:, None, None] * phase)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-7)


@pytest.mark.parametrize("model,N", [(oracle.FD_D2Q9, 2), (oracle.FD_D2Q16, 3), (oracle.FD_D2Q36, 4)])
def test_conservation_and_uniform_state(model, N):
    rng = np.random.default_rng(21)
    Nx, Ny = 9, 8
    ds = 1.0 / Nx
    tau = 1e-2
    dt = 0.5 * ds / 3.4
    sim = oracle.OracleSim(model, Nx, Ny, tau, dt, ds, N)
    sim.init(rng.uniform(0.9, 1.1, (Ny, Nx)), rng.uniform(-0.05, 0.05, (Ny, Nx)),
             rng.uniform(-0.05, 0.05, (Ny, Nx)))
    d0 = sim.reduce()
    sim.step(20)
    d1 = sim.reduce()
    tol = 20 * 3 * 64 * 2.0 ** -53 * d0[0]
    assert abs(d1[0] - d0[0]) <= tol
    assert abs(d1[1] - d0[1]) <= tol
    assert abs(d1[2] - d0[2]) <= tol
    assert d1[3] < d0[3]
    # uniform state: every node does the same arithmetic
    sim.init(np.full((Ny, Nx), 1.02), np.full((Ny, Nx), 0.03), np.full((Ny, Nx), -0.02))
    f0 = sim.get_state()
    sim.step(5)
    f1 = sim.get_state()
    for k in range(sim.K):
        assert np.all(f1[k] == f1[k, 0, 0])
    np.testing.assert_allclose(f1, f0, rtol=1e-13, atol=1e-16)


def test_shear_wave_viscosity_fd():
    """Shear wave u_y = U sin(2 pi x), FD D2Q16 (N = 3), nu_FD = tau_FD = 5e-4:
    the fitted viscosity approaches tau_FD with fifth-order spatial error."""
    U, tau = 0.01, 5e-4
    nus = {}
    for Nx in (16, 32):
        ds = 1.0 / Nx
        dt = 5e-4
        sim = oracle.OracleSim(oracle.FD_D2Q16, Nx, 1, tau, dt, ds, 3)
        x = np.arange(Nx)[None, :] * ds
        pat = np.sin(2 * np.pi * x)
        sim.init(np.ones((1, Nx)), np.zeros((1, Nx)), U * pat)
        t, a = [], []
        for n in range(0, 401, 20):
            if n:
                sim.step(20)
            if n >= 40:
                t.append(n * dt)
                a.append(sim.reduce(np.zeros_like(pat), pat)[4])
        nus[Nx] = exact.apparent_viscosity(t, a, 2 * np.pi, "shear")
    err16 = abs(nus[16] / tau - 1)
    err32 = abs(nus[32] / tau - 1)
    assert err32 < 0.01
    # order above 4.5 between 16 and 32 nodes (fifth-order WENO-5; measured 5.35)
    assert err16 / err32 > 2 ** 4.5


def test_fd_viscosity_linear_eigenvalue():
    """With the linear flux (eps -> inf) the shear decay per step is the
    eigenvalue of the linear one-step matrix."""
    Nx, tau, dt, U = 20, 5e-4, 5e-4, 0.01
    ds = 1.0 / Nx
    sim = oracle.OracleSim(oracle.FD_D2Q9, Nx, 1, tau, dt, ds, 2)
    sim.set_weno_eps(1e30)
    vx, vy, w = sim.velocities()
    x = np.arange(Nx)[None, :] * ds
    pat = np.sin(2 * np.pi * x)
    sim.init(np.ones((1, Nx)), np.zeros((1, Nx)), U * pat)
    t, a = [], []
    for n in range(0, 2001, 50):
        if n:
            sim.step(50)
        if n >= 200:
            t.append(n * dt)
            a.append(sim.reduce(np.zeros_like(pat), pat)[4])
    nu_fit = exact.apparent_viscosity(t, a, 2 * np.pi, "shear")
    q = np.array([2 * np.pi / Nx, 0.0])
    lam, vec = np.linalg.eig(linear_fd_matrix(q, ds, dt, tau, vx, vy, w))
    shear = w * vy
    overlap = np.abs(vec.conj().T @ shear) / np.linalg.norm(vec, axis=0)
    lam_s = lam[np.argmax(overlap)]
    nu_eig = -np.log(abs(lam_s)) / dt / (2 * np.pi) ** 2
    assert nu_fit == pytest.approx(nu_eig, rel=1e-7)


# ------------------------------------------------- Tables 1 and 2, FD column ---

def fd_table_error(kind, n, threads=1):
    """Relative error of the apparent viscosity of one FD entry of Table 1
    (shear wave, Section 4.2) or Table 2 (Taylor-Green vortex, Section 4.3):
    Gauss-Hermite D2Q9 (N = 2) on the unit box with n nodes per side,
    U = 0.01, k = 2 pi, nu_FD = tau_FD = dt = 5e-4 (the time step of
    Section 4.2), WENO eps = 1e-12 (far below the smoothness indicators, so
    the nonlinear weights are the pure Jiang-Shu ones), rho = 1 uniform;
    ln A(t) fitted over 0 <= t <= 2 with 400 samples."""
    U, tau = 0.01, 5e-4
    k = 2 * math.pi
    ny = 1 if kind == "shear" else n
    X, Y = np.meshgrid(np.arange(n) / n, np.arange(ny) / ny)
    if kind == "shear":
        px, py = np.zeros((ny, n)), np.sin(k * X)
    else:
        px, py = np.sin(k * X) * np.cos(k * Y), -np.cos(k * X) * np.sin(k * Y)
    sim = oracle.OracleSim(oracle.FD_D2Q9, n, ny, tau, tau, 1.0 / n, 2)
    sim.set_weno_eps(1e-12)
    sim.set_threads(threads)
    sim.init(np.ones((ny, n)), U * px, U * py)
    steps, every = 4000, 10
    t, a = [], []
    for s in range(0, steps + 1, every):
        if s:
            sim.step(every)
        t.append(s * tau)
        a.append(sim.reduce(px, py)[4])
    return exact.apparent_viscosity(np.array(t), np.array(a), k, kind) / tau - 1


def test_table1_fd_column(golden):
    """The FD column of Table 1 (shear-wave viscosity error, N = 20 .. 60)
    to its printed digits.  It depends on the WENO-5 nonlinear weights: a
    wrong coefficient in a smoothness indicator moves the N = 20 error by a
    factor of several."""
    g = golden("paper_tables.txt")
    ns = [int(v) for v in g["n"].split()]
    printed = [float(v) for v in g["shear_fd_err"].split()]
    got = [fd_table_error("shear", n) for n in ns]
    for n, e, p in zip(ns, got, printed):
        assert abs(e - p) <= 0.02 * p + 1.01e-4, (n, e, p)
    order = -np.polyfit(np.log(ns), np.log(np.abs(got)), 1)[0]
    assert order > 4.5


def test_table2_fd_column(golden):
    """The FD column of Table 2 (Taylor-Green vortex viscosity error) at
    N = 20 and 30, to its printed digits."""
    g = golden("paper_tables.txt")
    ns = [int(v) for v in g["n"].split()]
    printed = dict(zip(ns, [float(v) for v in g["tgv_fd_err"].split()]))
    threads = max(1, min(8, os.cpu_count() or 1))
    for n in (20, 30):
        e = fd_table_error("tgv", n, threads)
        assert abs(e - printed[n]) <= 0.02 * printed[n] + 1.01e-4, (n, e, printed[n])


# ------------------------------------------------------ row-parallel mode ---

@pytest.mark.parametrize("model,N,imex,fixed", [(oracle.CS_D2Q9, 2, False, False), (oracle.CS_D2Q9, 2, False, True),
                                                (oracle.FD_D2Q16, 3, False, False), (oracle.FD_D2Q9, 2, True, False),
                                                (oracle.FD_D2Q36, 4, False, True)])
def test_threads_bitwise(model, N, imex, fixed):
    """The row-parallel mode computes every node with the same operations:
    bitwise the single-threaded state."""
    Nx, Ny = 13, 11
    if model == oracle.CS_D2Q9:
        args = (0.7, 1.0, 1.0)
    else:
        ds = 1.0 / Nx
        dt = 0.4 * ds / 3.4
        args = (dt if imex else 2 * dt, dt, ds)
    rng = np.random.default_rng(31)
    rho, ux, uy = rng.uniform(0.9, 1.1, (Ny, Nx)), rng.uniform(-0.05, 0.05, (Ny, Nx)), rng.uniform(-0.05, 0.05, (Ny, Nx))
    out = []
    for threads in (1, 4):
        sim = oracle.OracleSim(model, Nx, Ny, *args, N)
        sim.set_threads(threads)
        if imex:
            sim.set_time_scheme(1)
        if fixed:
            sim.set_bc_x(1.05, 0.95)
        sim.init(rho, ux, uy)
        sim.step(3)
        out.append((sim.get_state(), sim.moments()))
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
