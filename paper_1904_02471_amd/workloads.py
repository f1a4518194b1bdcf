"""Seeded, synthetic initial states and request traces.

This module holds input generators only: closed-form initial fields
(shear wave, Taylor-Green vortex, shock tube, random states) and the
request trace of the serving stream.  It contains none of the lattice
Boltzmann arithmetic and is shared by the tests, the benchmark and users.

Node coordinates are x_i = i, y_j = j in node units (multiply by the grid
spacing for physical units); fields are returned as [Ny][Nx] float64.
"""
import math

import numpy as np


def grid(Nx, Ny):
    """Node index arrays X[j, i] = i, Y[j, i] = j."""
    return np.meshgrid(np.arange(Nx, dtype=np.float64), np.arange(Ny, dtype=np.float64))


def shear_wave(Nx, Ny, U, direction="y", rho0=1.0):
    """Transverse shear wave with one wavelength across the box.

    direction "y": u_x = U sin(2 pi y / Ny), u_y = 0   (wave vector along y)
    direction "x": u_y = U sin(2 pi x / Nx), u_x = 0   (wave vector along x)
    Returns rho, ux, uy and the velocity pattern (phi_x, phi_y) whose
    projection gives the amplitude."""
    X, Y = grid(Nx, Ny)
    rho = np.full((Ny, Nx), float(rho0))
    if direction == "y":
        px, py = np.sin(2 * math.pi * Y / Ny), np.zeros((Ny, Nx))
    elif direction == "x":
        px, py = np.zeros((Ny, Nx)), np.sin(2 * math.pi * X / Nx)
    else:
        raise ValueError(direction)
    return rho, U * px, U * py, (px, py)


def taylor_green(Nx, Ny, U, cs2, rho0=1.0, with_pressure=True):
    """Taylor-Green vortex with one period across the box (k = 2 pi / N):
    u_x = U sin(kx) cos(ky), u_y = -U cos(kx) sin(ky), and, when
    with_pressure, rho = rho0 - rho0 U^2 / (4 cs2) (cos 2kx + cos 2ky)."""
    X, Y = grid(Nx, Ny)
    kx, ky = 2 * math.pi / Nx, 2 * math.pi / Ny
    px = np.sin(kx * X) * np.cos(ky * Y)
    py = -np.cos(kx * X) * np.sin(ky * Y)
    rho = np.full((Ny, Nx), float(rho0))
    if with_pressure:
        rho = rho - rho0 * U * U / (4.0 * cs2) * (np.cos(2 * kx * X) + np.cos(2 * ky * Y))
    return rho, U * px, U * py, (px, py)


def separable_pattern(kind, Nx, Ny):
    """The same velocity patterns as products of 1-D factors:
    phi_x(i, j) = ax[i] * ay[j], phi_y(i, j) = bx[i] * by[j]."""
    x = np.arange(Nx, dtype=np.float64)
    y = np.arange(Ny, dtype=np.float64)
    kx, ky = 2 * math.pi / Nx, 2 * math.pi / Ny
    if kind == "shear_y":
        return np.ones(Nx), np.sin(ky * y), np.zeros(Nx), np.zeros(Ny)
    if kind == "shear_x":
        return np.zeros(Nx), np.zeros(Ny), np.sin(kx * x), np.ones(Ny)
    if kind == "tgv":
        return np.sin(kx * x), np.cos(ky * y), -np.cos(kx * x), np.sin(ky * y)
    raise ValueError(kind)


def shock_tube(Nx, Ny, rho_l, rho_r, width=None):
    """Density step at the middle of the box, u = 0.  width=None gives the
    sharp step (nodes i < Nx/2 hold rho_l); otherwise a tanh profile
    rho = (rho_l + rho_r)/2 - (rho_l - rho_r)/2 tanh((i - x0) / width) with
    x0 = Nx/2 - 1/2, antisymmetric about the middle between two nodes."""
    X, _ = grid(Nx, Ny)
    if width is None:
        rho = np.where(X < Nx // 2, float(rho_l), float(rho_r))
    else:
        x0 = Nx / 2.0 - 0.5
        rho = 0.5 * (rho_l + rho_r) - 0.5 * (rho_l - rho_r) * np.tanh((X - x0) / width)
    return rho, np.zeros((Ny, Nx)), np.zeros((Ny, Nx))


def random_state(Nx, Ny, seed, cs, rho_range=(0.9, 1.1), u_max=0.05):
    """rho ~ U[rho_range], u ~ U[-u_max, u_max] * cs, seeded (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(rho_range[0], rho_range[1], (Ny, Nx))
    ux = rng.uniform(-u_max, u_max, (Ny, Nx)) * cs
    uy = rng.uniform(-u_max, u_max, (Ny, Nx)) * cs
    return rho, ux, uy


def separable_random_state(Nx, Ny, seed, u_max=0.02, rho_spread=0.01):
    """A state that varies from node to node in both directions yet costs
    one full-size array per field (for grids of ~1e9 nodes):
    rho = 1 + rho_spread (a[i] + b[j]) / 2, u_x = u_max c[i] d[j],
    u_y = u_max e[i] f[j], the 1-D factors uniform in [-1, 1] (seeded).
    Returns rho, ux, uy and a function giving the three fields on the index
    window (ys, xs) without slicing the full arrays."""
    rng = np.random.default_rng(seed)
    a, c, e = (rng.uniform(-1.0, 1.0, Nx) for _ in range(3))
    b, d, f = (rng.uniform(-1.0, 1.0, Ny) for _ in range(3))

    def window(ys, xs):
        return (1.0 + 0.5 * rho_spread * np.add.outer(b[ys], a[xs]),
                u_max * np.multiply.outer(d[ys], c[xs]), u_max * np.multiply.outer(f[ys], e[xs]))

    rho = np.add.outer(b, a)
    rho *= 0.5 * rho_spread
    rho += 1.0
    ux = np.multiply.outer(d, c)
    ux *= u_max
    uy = np.multiply.outer(f, e)
    uy *= u_max
    return rho, ux, uy, window


def random_distribution(K, Nx, Ny, seed, weights, spread=0.2):
    """A non-equilibrium distribution: w_k (1 + spread * U[-1, 1])."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)[:, None, None]
    return w * (1.0 + spread * rng.uniform(-1.0, 1.0, (K, Ny, Nx)))


def serving_trace(n_requests=512, seed=1904, mean_gap_s=2e-3, sides=(64, 128, 256, 512, 1024),
                  tau_range=(0.55, 1.5), steps_range=(500, 5000), u0=0.01):
    """Request stream: exponential inter-arrival gaps (Poisson arrivals),
    kind shear/TGV 50/50, square side uniform over `sides`, model CS D2Q9 or
    FD D2Q16 50/50, CS relaxation time uniform in tau_range (standard lattice
    units), steps uniform in steps_range.  Deterministic for a seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(mean_gap_s)
        out.append({
            "id": i,
            "arrival_s": t,
            "kind": "shear" if rng.random() < 0.5 else "tgv",
            "side": int(sides[rng.integers(len(sides))]),
            "model": "cs" if rng.random() < 0.5 else "fd16",
            "tau_std": float(rng.uniform(*tau_range)),
            "steps": int(rng.integers(steps_range[0], steps_range[1] + 1)),
            "u0": u0,
        })
    return out
