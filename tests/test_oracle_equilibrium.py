"""Pins of the oracle's equilibrium and moments (Section 1: the Hermite
coefficients are the velocity moments, and the quadrature reproduces the
moments of the equilibrium up to order N; Section 2: second-order form and
discrete moments)."""
import math

import numpy as np
import pytest

import oracle


def gaussian_moment(j):
    return 0.0 if j % 2 else float(math.prod(range(j - 1, 0, -2)) if j > 1 else 1.0)


def maxwellian_moment_1d(u, cs, a):
    # E[(u + cs Z)^a] by the binomial expansion
    return sum(math.comb(a, j) * u ** (a - j) * cs ** j * gaussian_moment(j) for j in range(a + 1))


CASES = [(oracle.CS_D2Q9, 2, (1.0, 1.0)), (oracle.CS_D2Q9, 2, (1.0, 1.0 / math.sqrt(3))),
         (oracle.CS_D2Q9, 2, (0.5, 0.2))]
for _model, _Q in [(oracle.FD_D2Q9, 3), (oracle.FD_D2Q16, 4), (oracle.FD_D2Q25, 5), (oracle.FD_D2Q36, 6)]:
    for _N in range(1, _Q):
        CASES.append((_model, _N, (0.01, 1e-3)))


@pytest.mark.parametrize("model,N,dsdt", CASES)
def test_equilibrium_moments_match_maxwellian(model, N, dsdt):
    ds, dt = dsdt
    sim = oracle.OracleSim(model, 4, 4, 1.0, dt, ds, N)
    vx, vy, w = sim.velocities()
    cs = sim.cs
    rng = np.random.default_rng(1904 + 31 * model + N)
    for _ in range(5):
        rho = rng.uniform(0.5, 1.5)
        ux, uy = rng.uniform(-0.3, 0.3, 2) * cs
        feq = sim.equilibrium(rho, ux, uy)
        for a in range(N + 1):
            for b in range(N + 1 - a):
                got = np.sum(feq * vx ** a * vy ** b)
                want = rho * maxwellian_moment_1d(ux, cs, a) * maxwellian_moment_1d(uy, cs, b)
                scale = rho * (abs(cs) + abs(ux) + abs(uy)) ** (a + b)
                assert abs(got - want) <= 1e-13 * scale, (model, N, a, b, got, want)


def test_truncation_is_real():
    # with N = 2 on a 16-velocity set, the third moment misses the u^3 term
    sim = oracle.OracleSim(oracle.FD_D2Q16, 4, 4, 1.0, 1e-3, 0.01, 2)
    vx, vy, w = sim.velocities()
    rho, ux, uy = 1.0, 0.2, 0.0
    feq = sim.equilibrium(rho, ux, uy)
    got = np.sum(feq * vx ** 3)
    want = maxwellian_moment_1d(ux, 1.0, 3)
    assert abs(got - want) == pytest.approx(ux ** 3, rel=1e-10)
    sim3 = oracle.OracleSim(oracle.FD_D2Q16, 4, 4, 1.0, 1e-3, 0.01, 3)
    assert abs(np.sum(sim3.equilibrium(rho, ux, uy) * vx ** 3) - want) < 1e-14


def test_init_then_moments_roundtrip():
    rng = np.random.default_rng(7)
    for model, N in [(oracle.CS_D2Q9, 2), (oracle.FD_D2Q16, 3), (oracle.FD_D2Q36, 4)]:
        sim = oracle.OracleSim(model, 5, 3, 0.8, 1.0 if model == 0 else 1e-3, 1.0 if model == 0 else 0.2, N)
        rho = rng.uniform(0.9, 1.1, (3, 5))
        ux = rng.uniform(-0.05, 0.05, (3, 5)) * sim.cs
        uy = rng.uniform(-0.05, 0.05, (3, 5)) * sim.cs
        sim.init(rho, ux, uy)
        r, x, y = sim.moments()
        np.testing.assert_allclose(r, rho, rtol=1e-14)
        np.testing.assert_allclose(x, ux, rtol=0, atol=1e-14)
        np.testing.assert_allclose(y, uy, rtol=0, atol=1e-14)
        # moments by their definition, from the state itself
        f = sim.get_state()
        vx, vy, _ = sim.velocities()
        np.testing.assert_allclose(f.sum(0), rho, rtol=1e-14)
        np.testing.assert_allclose(np.tensordot(vx, f, 1) / f.sum(0), ux, atol=1e-14)


def test_reduce_of_initial_state():
    rng = np.random.default_rng(11)
    sim = oracle.OracleSim(oracle.CS_D2Q9, 6, 4, 0.8, 1.0, 1.0, 2)
    rho = rng.uniform(0.9, 1.1, (4, 6))
    ux = rng.uniform(-0.02, 0.02, (4, 6))
    uy = rng.uniform(-0.02, 0.02, (4, 6))
    px, py = rng.standard_normal((2, 4, 6))
    sim.init(rho, ux, uy)
    out = sim.reduce(px, py)
    assert out[0] == pytest.approx(rho.sum(), rel=1e-14)
    assert out[1] == pytest.approx((rho * ux).sum(), rel=1e-12)
    assert out[2] == pytest.approx((rho * uy).sum(), rel=1e-12)
    assert out[3] == pytest.approx((0.5 * rho * (ux ** 2 + uy ** 2)).sum(), rel=1e-12)
    assert out[4] == pytest.approx((ux * px + uy * py).sum() / (px ** 2 + py ** 2).sum(), rel=1e-12)
    assert sim.reduce()[4] == 0.0
