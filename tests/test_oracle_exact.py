"""Pins of the exact solutions and conversions the oracle is judged by:
the isothermal Riemann problem (Section 4.1), the decay-law fit (Sections
4.2-4.3) and the FD/CS unit relations (Section 3)."""
import math

import numpy as np
import pytest

from oracle import exact


def half_unit(text):
    """Half a unit in the last printed digit of a decimal literal (a figure
    rounded to the digits shown)."""
    mant = text.lower().split("e")[0]
    exp = int(text.lower().split("e")[1]) if "e" in text.lower() else 0
    dec = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (-dec + exp)


def test_printed_shock_example(golden):
    g = golden("shock_tube_example.txt")
    s = exact.riemann_solution(float(g["rho_l"]), float(g["rho_r"]), float(g["cs"]))
    # the printed figures are rounded (xi_c, rho_c) or truncated (zeta, u_c)
    # to the digits shown: allow one unit in the last digit
    for key in ("zeta", "xi_r", "xi_c", "u_c", "rho_c", "xi_s"):
        assert abs(s[key] - float(g[key])) <= 2 * half_unit(g[key]), (key, s[key], g[key])
    assert truncated(s["zeta"], 5) == pytest.approx(float(g["zeta"]), abs=1e-12)


@pytest.mark.parametrize("rl,rr,cs", [(1.1, 0.9, 1.0), (1.5, 1.0, 1.0), (2.0, 0.5, 0.7), (1.5, 1.0, 1 / math.sqrt(3))])
def test_rankine_hugoniot_and_fan(rl, rr, cs):
    s = exact.riemann_solution(rl, rr, cs)
    rc, uc, xs = s["rho_c"], s["u_c"], s["xi_s"]
    # mass and momentum fluxes continuous across the shock (P = rho c_s^2)
    assert rc * (uc - xs) == pytest.approx(rr * (0.0 - xs), rel=1e-12)
    assert rc * uc * (uc - xs) + rc * cs ** 2 == pytest.approx(rr * cs ** 2, rel=1e-12)
    # the fan joins the left state at xi_r and the plateau at xi_c
    rho, u = exact.riemann_profile(np.array([s["xi_r"], s["xi_c"] - 1e-13]), rl, rr, cs)
    assert rho[0] == pytest.approx(rl, rel=1e-12) and abs(u[0]) < 1e-12
    assert rho[1] == pytest.approx(rc, rel=1e-10) and u[1] == pytest.approx(uc, rel=1e-10)
    # the fan satisfies the similarity equations du/dxi = (xi-u)/rho drho/dxi
    # and dP/dxi = (xi-u)^2 drho/dxi
    xi = np.linspace(s["xi_r"] + 1e-3, s["xi_c"] - 1e-3, 50)
    h = 1e-6
    rp, up = exact.riemann_profile(xi + h, rl, rr, cs)
    rm, um = exact.riemann_profile(xi - h, rl, rr, cs)
    r0, u0 = exact.riemann_profile(xi, rl, rr, cs)
    drho, du = (rp - rm) / (2 * h), (up - um) / (2 * h)
    np.testing.assert_allclose(du, (xi - u0) / r0 * drho, rtol=1e-7)
    np.testing.assert_allclose(cs ** 2 * drho, (xi - u0) ** 2 * drho, rtol=1e-7)


def test_zeta_is_the_unique_root():
    for rl, rr in [(1.1, 0.9), (1.5, 1.0), (3.0, 1.0)]:
        z = exact.riemann_zeta(rl, rr)
        r = rl / rr
        g = lambda x: 2 + x * x - r * math.exp(-x) - math.exp(x) / r
        assert abs(g(z)) < 1e-14
        grid = np.linspace(1e-9, math.log(r), 2001)
        vals = np.array([g(x) for x in grid])
        assert np.sum(np.diff(np.sign(vals)) != 0) == 1


def test_fit_recovers_exact_exponentials():
    t = np.linspace(0, 3, 40)
    assert exact.fit_decay_rate(t, 0.01 * np.exp(-0.37 * t)) == pytest.approx(0.37, rel=1e-13)
    k, nu = 2 * math.pi, 5e-4
    assert exact.apparent_viscosity(t, exact.shear_amplitude(0.01, k, nu, t), k, "shear") == pytest.approx(nu, rel=1e-12)
    assert exact.apparent_viscosity(t, exact.taylor_green_amplitude(0.01, k, nu, t), k, "tgv") == pytest.approx(nu, rel=1e-12)


def test_acoustic_fit_separates_a_ringing_sound_wave():
    # a slow vortex decaying by 4e-4 over the window, modulated 1e-4 by a
    # standing sound wave at 2 k c_s: the plain fit is biased by percents,
    # the fit with the modulation recovers the rate
    n, nu, cs = 4096, 0.05 / 3, 1 / math.sqrt(3)
    k = 2 * math.pi / n
    t = np.arange(0, 5001, 10.0)
    omega = 2 * k * cs
    amp = 0.01 * np.exp(-2 * k * k * nu * t) * (1 + 1e-4 * np.cos(omega * t + 0.7))
    assert abs(exact.apparent_viscosity(t, amp, k, "tgv") / nu - 1) > 1e-2
    assert exact.apparent_viscosity(t, amp, k, "tgv", omega=omega) == pytest.approx(nu, rel=1e-5)
    clean = 0.01 * np.exp(-2 * k * k * nu * t)
    assert exact.apparent_viscosity(t, clean, k, "tgv", omega=omega) == pytest.approx(nu, rel=1e-9)


def truncated(x, digits):
    return math.floor(x * 10 ** digits + 1e-9) / 10 ** digits


def test_printed_relaxation_times(golden):
    g = golden("tau_conversion.txt")
    n = int(g["shock_n"])
    for key in ("a", "b"):
        printed = g["shock_tau_lu_" + key]
        digits = len(printed.split(".")[1])
        got = exact.tau_lu_from_fd(float(g["shock_tau_fd_" + key]), n)
        assert truncated(got, digits) == pytest.approx(float(printed), abs=1e-12)
    tau_fd = float(g["table_tau_fd"])
    for n, printed in zip(g["table_n"].split(), g["table_tau_lu"].split()):
        got = exact.tau_lu_from_fd(tau_fd, int(n))
        assert truncated(got, 4) == pytest.approx(float(printed), abs=1e-12)
        # and the inverse relation
        assert exact.tau_fd_from_lu(got, int(n)) == pytest.approx(tau_fd, rel=1e-12)
        # same viscosity: nu_LU = N nu_FD
        assert exact.nu_lu(got) == pytest.approx(int(n) * tau_fd, rel=1e-12)


def test_printed_time_steps(golden):
    g = golden("time_steps.txt")
    n = int(g["n"])
    dt = exact.cs_dt_in_fd_units(n)
    assert abs(dt - float(g["dt_cs_fd"])) <= half_unit(g["dt_cs_fd"])
    assert abs(dt / 3 - float(g["dt_fd_reduced"])) <= half_unit(g["dt_fd_reduced"])
    t_cs = int(g["cs_iterations"]) * dt
    t_fd = int(g["fd_iterations_reduced"]) * dt / 3
    assert abs(t_cs - float(g["t_final"])) <= half_unit(g["t_final"])
    assert t_fd == pytest.approx(t_cs, rel=1e-12)
    # Section 4.2: the CS step is about 5e-4 * (1155 / N) in FD units
    for nx in (20, 40, 60):
        assert exact.cs_dt_in_fd_units(nx) == pytest.approx(float(g["shear_dt_fd"]) * int(g["shear_factor"]) / nx,
                                                           rel=1e-3)


def test_standard_lattice_units_bridge():
    # tau_std = sqrt(3) tau_LU, and both give the same FD viscosity
    for n in (64, 512, 2048):
        for tau_std in (0.55, 0.6, 0.8, 1.5):
            tau_fd = exact.tau_fd_from_std(tau_std, n)
            tau_lu = exact.tau_lu_from_fd(tau_fd, n)
            assert exact.tau_std_from_lu(tau_lu) == pytest.approx(tau_std, rel=1e-13)
    assert exact.tau_fd_from_std(0.6, 512) == pytest.approx(1.12764e-4, rel=1e-5)
