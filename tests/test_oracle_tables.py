"""Pins of the oracle's velocity sets (Section 1: Gauss-Hermite quadrature;
Section 2: the CS D2Q9 lattice with |v_k,alpha| = c_l = ds/dt)."""
import math

import numpy as np
import pytest

import oracle


def double_factorial(n):
    return 1 if n <= 0 else n * double_factorial(n - 2)


@pytest.mark.parametrize("Q", [2, 3, 4, 5, 6, 7, 8])
def test_quadrature_moments_exact(Q):
    # Gauss rule with Q nodes integrates x^n exactly for n <= 2Q-1:
    # E[Z^n] = (n-1)!! for even n, 0 for odd n (Z standard normal).
    x, w = oracle.gauss_hermite(Q)
    for n in range(2 * Q):
        exact = 0.0 if n % 2 else float(double_factorial(n - 1))
        got = np.sum(w * x ** n)
        scale = np.sum(w * np.abs(x) ** n)   # size of the terms summed
        assert abs(got - exact) <= 1e-14 * max(1.0, scale), (Q, n, got, exact)
    # and not for n = 2Q (the rule has degree exactly 2Q-1)
    assert abs(np.sum(w * x ** (2 * Q)) - double_factorial(2 * Q - 1)) > 1e-6


def test_closed_form_roots():
    # He_2 = x^2-1, He_3 = x^3-3x, He_4 = x^4-6x^2+3, He_5 = x^5-10x^3+15x
    x, w = oracle.gauss_hermite(2)
    np.testing.assert_allclose(x, [-1, 1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], rtol=0, atol=1e-15)
    x, w = oracle.gauss_hermite(3)
    np.testing.assert_allclose(x, [-math.sqrt(3), 0, math.sqrt(3)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=0, atol=1e-15)
    x, _ = oracle.gauss_hermite(4)
    a, b = math.sqrt(3 - math.sqrt(6)), math.sqrt(3 + math.sqrt(6))
    np.testing.assert_allclose(x, [-b, -a, a, b], rtol=0, atol=1e-14)
    x, _ = oracle.gauss_hermite(5)
    a, b = math.sqrt(5 - math.sqrt(10)), math.sqrt(5 + math.sqrt(10))
    np.testing.assert_allclose(x, [-b, -a, 0, a, b], rtol=0, atol=1e-14)


@pytest.mark.parametrize("Q", [2, 3, 4, 5, 6, 7, 8])
def test_against_numpy_hermegauss(Q):
    # library routine for the same rule (weights normalised to sum 1)
    xr, wr = np.polynomial.hermite_e.hermegauss(Q)
    wr = wr / wr.sum()
    x, w = oracle.gauss_hermite(Q)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w, wr, rtol=1e-12, atol=0)


def test_d2q9_cs_lattice():
    ds, dt = 1.0, 1.0 / math.sqrt(3.0)       # the paper's CS units
    vx, vy, w, cs = oracle.velocity_set(oracle.CS_D2Q9, ds, dt)
    cl = ds / dt
    assert cs == pytest.approx(1.0, abs=1e-15)  # c_s = 1 in the paper's LU
    # order: rest, E, N, W, S, NE, NW, SW, SE
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    np.testing.assert_allclose(vx, e[:, 0] * cl, atol=1e-15)
    np.testing.assert_allclose(vy, e[:, 1] * cl, atol=1e-15)
    np.testing.assert_allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)
    # standard lattice units: c_s^2 = 1/3
    _, _, _, cs1 = oracle.velocity_set(oracle.CS_D2Q9, 1.0, 1.0)
    assert cs1 ** 2 == pytest.approx(1 / 3, rel=1e-15)


@pytest.mark.parametrize("model,Q", [(oracle.FD_D2Q9, 3), (oracle.FD_D2Q16, 4), (oracle.FD_D2Q25, 5),
                                     (oracle.FD_D2Q36, 6)])
def test_fd_tensor_sets(model, Q):
    vx, vy, w, cs = oracle.velocity_set(model)
    x, wq = oracle.gauss_hermite(Q)
    assert cs == 1.0 and len(vx) == Q * Q
    for j in range(Q):
        for i in range(Q):
            k = j * Q + i
            assert vx[k] == x[i] and vy[k] == x[j] and w[k] == pytest.approx(wq[i] * wq[j], rel=1e-15)
    assert np.sum(w) == pytest.approx(1.0, abs=1e-14)
