"""Pins of the oracle's collision-streaming step (Section 2, CS evolution
equation f_k(x + v_k dt, t + dt) - f_k(x, t) = -(dt/tau)(f_k - f_eq_k), and
the CS viscosity nu = c_s^2 (tau - dt/2))."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact

E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])


def linear_cs_matrix(q, omega, w, xi):
    """One CS step linearised at rho = 1, u = 0 for the Fourier mode
    exp(i q.x): a' = S [(1 - omega) I + omega Eq] a, with the equilibrium
    Jacobian Eq_kl = w_k (1 + xi_k . xi_l) and the shift S_kk = exp(-i q.e_k)
    (value at x comes from x - e_k)."""
    K = len(w)
    Eq = w[:, None] * (1.0 + xi @ xi.T)
    S = np.diag(np.exp(-1j * (E @ q)))
    return S @ ((1 - omega) * np.eye(K) + omega * Eq)


def central_difference(sim, w, pert, eps=1e-6):
    """(step(w + eps p) - step(w - eps p)) / (2 eps): the linear response of
    one step about the rest state, free of the quadratic terms."""
    out = []
    for sgn in (1.0, -1.0):
        sim.set_state(w[:, None, None] + sgn * eps * pert)
        sim.step(1)
        out.append(sim.get_state())
    return (out[0] - out[1]) / (2 * eps)


@pytest.mark.parametrize("tau,dsdt", [(0.8, (1.0, 1.0)), (0.55, (1.0, 1.0)), (0.4, (1.0, 1 / math.sqrt(3)))])
def test_linear_response_one_step(tau, dsdt):
    ds, dt = dsdt
    Nx, Ny = 12, 10
    sim = oracle.OracleSim(oracle.CS_D2Q9, Nx, Ny, tau, dt, ds, 2)
    vx, vy, w = sim.velocities()
    xi = np.stack([vx, vy], 1) / sim.cs
    rng = np.random.default_rng(3)
    for m, n in [(1, 0), (0, 1), (2, 3), (5, 4)]:
        q = 2 * np.pi * np.array([m / Nx, n / Ny])
        a = rng.standard_normal(9) + 1j * rng.standard_normal(9)
        X, Y = np.meshgrid(np.arange(Nx), np.arange(Ny))
        phase = np.exp(1j * (q[0] * X + q[1] * Y))
        got = central_difference(sim, w, np.real(a[:, None, None] * phase))
        a1 = linear_cs_matrix(q, dt / tau, w, xi) @ a
        want = np.real(a1[:, None, None] * phase)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-8)


def test_full_relaxation_streams_equilibrium():
    # omega = 1: the post-collision state is f_eq of the node, moved one link
    rng = np.random.default_rng(5)
    Nx, Ny = 7, 5
    sim = oracle.OracleSim(oracle.CS_D2Q9, Nx, Ny, 1.0, 1.0, 1.0, 2)
    f = rng.uniform(0.01, 0.3, (9, Ny, Nx))
    sim.set_state(f)
    vx, vy, _ = sim.velocities()
    rho = f.sum(0)
    ux = np.tensordot(vx, f, 1) / rho
    uy = np.tensordot(vy, f, 1) / rho
    sim.step(1)
    got = sim.get_state()
    for k in range(9):
        feq = np.array([[sim.equilibrium(rho[y, x], ux[y, x], uy[y, x])[k] for x in range(Nx)] for y in range(Ny)])
        want = np.roll(feq, shift=(E[k, 1], E[k, 0]), axis=(0, 1))
        np.testing.assert_allclose(got[k], want, rtol=1e-14, atol=0)


def test_conservation_periodic():
    rng = np.random.default_rng(9)
    Nx, Ny = 11, 9
    sim = oracle.OracleSim(oracle.CS_D2Q9, Nx, Ny, 0.6, 1.0, 1.0, 2)
    sim.init(rng.uniform(0.9, 1.1, (Ny, Nx)), rng.uniform(-0.05, 0.05, (Ny, Nx)),
             rng.uniform(-0.05, 0.05, (Ny, Nx)))
    d0 = sim.reduce()
    sim.step(300)
    d1 = sim.reduce()
    # rounding only: a few units of 2^-53 per step (the weights sum to 1 only
    # to the last bit, so the drift is systematic, not a random walk)
    tol = 300 * 16 * 2.0 ** -53 * d0[0]
    assert abs(d1[0] - d0[0]) <= tol
    assert abs(d1[1] - d0[1]) <= tol
    assert abs(d1[2] - d0[2]) <= tol
    assert d1[3] < d0[3]   # kinetic energy is dissipated


def test_uniform_state_stays_uniform():
    sim = oracle.OracleSim(oracle.CS_D2Q9, 6, 5, 0.7, 1.0, 1.0, 2)
    sim.init(np.full((5, 6), 1.03), np.full((5, 6), 0.02), np.full((5, 6), -0.01))
    f0 = sim.get_state()
    sim.step(50)
    f1 = sim.get_state()
    for k in range(9):
        assert np.all(f1[k] == f1[k, 0, 0])       # bitwise uniform
    np.testing.assert_allclose(f1, f0, rtol=50 * 8 * 2.0 ** -53)  # rounding only


def shear_run(sim, U, steps, every=1):
    Ny, Nx = sim.Ny, sim.Nx
    y = np.arange(Ny)[:, None] * np.ones((1, Nx))
    pat = np.sin(2 * np.pi * y / Ny)
    sim.init(np.ones((Ny, Nx)), U * pat, np.zeros((Ny, Nx)))
    t, a, e = [0.0], [sim.reduce(pat, np.zeros_like(pat))[4]], [sim.reduce()[3]]
    for n in range(every, steps + 1, every):
        sim.step(every)
        out = sim.reduce(pat, np.zeros_like(pat))
        t.append(n * sim.dt)
        a.append(out[4])
        e.append(out[3])
    return np.array(t), np.array(a), np.array(e)


def test_shear_wave_decay_matches_linear_eigenvalue():
    """64x64, tau = 0.8, ds = dt = 1, u_x = 1e-3 sin(2 pi y / 64), 1000 steps.
    The decay per step of the shear mode is the eigenvalue of the linear
    one-step operator; the analytic viscosity (tau - 1/2)/3 = 0.1 differs
    from it by the lattice error only."""
    N = 64
    sim = oracle.OracleSim(oracle.CS_D2Q9, N, N, 0.8, 1.0, 1.0, 2)
    t, a, e = shear_run(sim, 1e-3, 1000, every=10)
    vx, vy, w = sim.velocities()
    xi = np.stack([vx, vy], 1) / sim.cs
    q = np.array([0.0, 2 * np.pi / N])
    lam, vec = np.linalg.eig(linear_cs_matrix(q, 1.0 / 0.8, w, xi))
    shear = w * xi[:, 0]                                   # x-momentum mode
    overlap = np.abs(vec.conj().T @ shear) / np.linalg.norm(vec, axis=0)
    lam_s = lam[np.argmax(overlap)]
    nu_eig = -np.log(abs(lam_s)) / (q[1] ** 2)
    sel = t >= 50
    nu_fit = exact.apparent_viscosity(t[sel], a[sel], q[1], "shear")
    assert nu_fit == pytest.approx(nu_eig, rel=1e-5)
    assert nu_eig == pytest.approx(0.1000514, abs=2e-7)
    assert nu_fit == pytest.approx(0.1, rel=1e-3)          # lattice error ~5e-4
    # kinetic energy decays at twice the amplitude rate
    gam_e = exact.fit_decay_rate(t[sel], e[sel])
    assert gam_e / (2 * q[1] ** 2) == pytest.approx(nu_eig, rel=1e-4)
    # amplitude ratio between step 100 and step 1000 is |lambda|^900; the
    # initial equilibrium start adds a transient of relative size ~5e-4
    assert a[-1] / a[10] == pytest.approx(abs(lam_s) ** 900, rel=1e-6)
    assert a[-1] / a[0] == pytest.approx(abs(lam_s) ** 1000, rel=1e-3)
