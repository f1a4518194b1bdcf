"""Closed-form results the oracle is checked against, and the host-side
analysis of its output (test infrastructure).

* Exact solution of the isothermal Riemann problem (Section 4.1).
* Decay laws of shear waves and Taylor-Green vortices (Sections 4.2, 4.3).
* Least-squares fit of the apparent viscosity (Sections 4.2, 4.3).
* Relations between the FD and CS non-dimensionalisations (Section 3).
"""
import math

import numpy as np

SQRT3 = math.sqrt(3.0)


# --------------------------------------------------------------------------
# Exact isothermal Riemann problem, rho_L > rho_R, u_L = u_R = 0 (Section 4.1)
# --------------------------------------------------------------------------

def riemann_zeta(rho_l, rho_r):
    """Root zeta in (0, ln(rho_l/rho_r)] of
    2 + z^2 - (rho_l/rho_r) e^{-z} - (rho_r/rho_l) e^{z} = 0 (Section 4.1),
    found by bisection: the left end is negative (r + 1/r > 2) and the right
    end equals ln(r)^2 > 0."""
    if not rho_l > rho_r > 0:
        raise ValueError("need rho_l > rho_r > 0")
    r = rho_l / rho_r

    def g(z):
        return 2.0 + z * z - r * math.exp(-z) - math.exp(z) / r

    lo, hi = 0.0, math.log(r)
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        if g(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def riemann_solution(rho_l, rho_r, cs=1.0):
    """Characteristic speeds and plateau state of the isothermal Riemann
    problem: head of the rarefaction xi_r = -c_s, its tail
    xi_c = c_s (zeta - 1), plateau u_c = zeta c_s, rho_c = rho_l e^{-zeta},
    shock speed xi_s = zeta c_s / (1 - (rho_r/rho_l) e^{zeta})."""
    z = riemann_zeta(rho_l, rho_r)
    return {
        "zeta": z,
        "xi_r": -cs,
        "xi_c": cs * (z - 1.0),
        "u_c": z * cs,
        "rho_c": rho_l * math.exp(-z),
        "xi_s": z * cs / (1.0 - (rho_r / rho_l) * math.exp(z)),
    }


def riemann_profile(xi, rho_l, rho_r, cs=1.0):
    """rho(xi), u(xi) of the similarity solution, xi = (x - x0)/t.
    In the fan u = xi + c_s and rho = rho_l exp(-u/c_s) (the second form of
    the printed fan density; the first form carries a sign slip)."""
    s = riemann_solution(rho_l, rho_r, cs)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    left = xi < s["xi_r"]
    fan = (xi >= s["xi_r"]) & (xi < s["xi_c"])
    plateau = (xi >= s["xi_c"]) & (xi < s["xi_s"])
    right = xi >= s["xi_s"]
    rho[left], u[left] = rho_l, 0.0
    u[fan] = xi[fan] + cs
    rho[fan] = rho_l * np.exp(-u[fan] / cs)
    rho[plateau], u[plateau] = s["rho_c"], s["u_c"]
    rho[right], u[right] = rho_r, 0.0
    return rho, u


# --------------------------------------------------------------------------
# Decay laws and the viscosity fit (Sections 4.2, 4.3)
# --------------------------------------------------------------------------

def shear_amplitude(U, k, nu, t):
    """u~(t) = U exp(-k^2 nu t) (Section 4.2)."""
    return U * np.exp(-k * k * nu * np.asarray(t, dtype=np.float64))


def taylor_green_amplitude(U, k, nu, t):
    """u~(t) = U exp(-2 k^2 nu t) for k = (k, k) (Section 4.3)."""
    return U * np.exp(-2.0 * k * k * nu * np.asarray(t, dtype=np.float64))


def fit_decay_rate(t, amp):
    """Ordinary least-squares slope of ln|amp| against t; returns the decay
    rate gamma with amp ~ exp(-gamma t).  READING: the paper does not state
    its fit; this is the plain log-linear least-squares fit."""
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.abs(np.asarray(amp, dtype=np.float64)))
    tm, ym = t.mean(), y.mean()
    slope = np.sum((t - tm) * (y - ym)) / np.sum((t - tm) ** 2)
    return -slope


def fit_decay_rate_acoustic(t, amp, omega):
    """Decay rate gamma from a least-squares fit of
        ln|amp| = c - gamma t + a cos(omega t) + b sin(omega t).
    READING: a Taylor-Green vortex started from f = f_eq with the
    incompressible pressure is not an exact state of the isothermal lattice
    gas; the O(Ma^2) mismatch rings as a standing sound wave at wavevector
    (2k, 0) and (0, 2k), of frequency omega = 2 k c_s, which modulates the
    projection onto the vortex at the 1e-4 level.  Where the total decay of a
    run is of that size (a slow vortex on a large grid) the plain log-linear
    fit is biased by it, so the modulation is fitted along."""
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.abs(np.asarray(amp, dtype=np.float64)))
    X = np.stack([np.ones_like(t), -t, np.cos(omega * t), np.sin(omega * t)], 1)
    coef = np.linalg.lstsq(X, y, rcond=None)[0]
    return coef[1]


def apparent_viscosity(t, amp, k, kind, omega=None):
    """nu_app from a fit of the decay law: gamma/k^2 for a shear wave,
    gamma/(2 k^2) for a Taylor-Green vortex with k = (k, k).  With `omega`
    the acoustic modulation of that frequency is fitted along."""
    g = fit_decay_rate(t, amp) if omega is None else fit_decay_rate_acoustic(t, amp, omega)
    if kind == "shear":
        return g / (k * k)
    if kind == "tgv":
        return g / (2.0 * k * k)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Non-dimensionalisation (Section 3).  "Paper lattice units" (LU): ds = 1,
# dt = 1/sqrt(3), c_s = 1.  FD units: length L = 1, c_s = 1.
# --------------------------------------------------------------------------

def tau_lu_from_fd(tau_fd, n_lu):
    """tau_LU = N_LU tau_FD + sqrt(3)/6 (Section 3, viscosity transfer)."""
    return n_lu * tau_fd + SQRT3 / 6.0


def tau_fd_from_lu(tau_lu, n_lu):
    return (tau_lu - SQRT3 / 6.0) / n_lu


def nu_lu(tau_lu, dt_lu=1.0 / SQRT3):
    """CS viscosity nu_LU = tau_LU - dt/2 (Section 2, c_s = 1)."""
    return tau_lu - dt_lu / 2.0


def cs_dt_in_fd_units(n_lu):
    """One CS step (dt_LU = 1/sqrt 3) in FD time units: t_ref,LU = t_ref,FD/N."""
    return 1.0 / (n_lu * SQRT3)


def tau_std_from_lu(tau_lu):
    """Standard lattice units (ds = dt = 1, c_s^2 = 1/3) share the length unit
    of the paper's LU; their time unit is one step, sqrt(3) times shorter."""
    return SQRT3 * tau_lu


def tau_fd_from_std(tau_std, n):
    """FD relaxation time matching a CS run at tau_std (ds = dt = 1) on n
    nodes: nu_std = (tau_std - 1/2)/3, nu_LU = sqrt(3) nu_std, nu_FD = nu_LU/n."""
    return (tau_std - 0.5) / (SQRT3 * n)
