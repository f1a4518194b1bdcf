"""CPU checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-side logic (velocity tables, parameter
validation, unit relations) is right.  No compute call needs a GPU here."""
import math
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT

from paper_1904_02471_amd import lb, units


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lb._lib, n), n
    assert sorted(lb.EXPORTS) == names


def test_library_is_built_for_gfx950():
    data = open(lb.LIB_PATH, "rb").read()
    assert b"gfx950" in data


@pytest.mark.parametrize("model,Q", [(lb.LB_FD_D2Q9, 3), (lb.LB_FD_D2Q16, 4), (lb.LB_FD_D2Q25, 5), (lb.LB_FD_D2Q36, 6)])
def test_model_tables_match_library_rule(model, Q):
    xr, wr = np.polynomial.hermite_e.hermegauss(Q)
    wr = wr / wr.sum()
    vx, vy, w, cs = lb.lb_model_info(model)
    assert cs == 1.0
    for j in range(Q):
        for i in range(Q):
            k = j * Q + i
            assert vx[k] == pytest.approx(xr[i], abs=1e-14)
            assert vy[k] == pytest.approx(xr[j], abs=1e-14)
            assert w[k] == pytest.approx(wr[i] * wr[j], rel=1e-13)
    # odd rules keep an exact zero velocity
    if Q % 2:
        assert vx[Q // 2] == 0.0


def test_d2q9_tables():
    vx, vy, w, cs = lb.lb_model_info(lb.LB_CS_D2Q9, 1.0, 1.0 / math.sqrt(3))
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    np.testing.assert_allclose(vx, e[:, 0] * math.sqrt(3), atol=1e-15)
    np.testing.assert_allclose(vy, e[:, 1] * math.sqrt(3), atol=1e-15)
    np.testing.assert_allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-15)
    assert cs == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("args,code", [
    ((lb.LB_CS_D2Q9, 8, 8, 0.4, 1.0, 1.0, 2), lb.LB_EINVAL),    # tau <= dt/2: negative viscosity
    ((lb.LB_CS_D2Q9, 8, 8, 0.8, 1.0, 1.0, 3), lb.LB_EINVAL),    # CS needs N = 2
    ((lb.LB_CS_D2Q9, 0, 8, 0.8, 1.0, 1.0, 2), lb.LB_EINVAL),    # empty grid
    ((lb.LB_FD_D2Q16, 8, 8, 1e-3, 1e-3, 0.1, 4), lb.LB_EINVAL),  # N > Q - 1
    ((lb.LB_FD_D2Q16, 8, 8, 1e-3, 1e-3, 0.1, 0), lb.LB_EINVAL),
    ((lb.LB_FD_D2Q16, 8, 8, 1.0, 0.05, 0.1, 3), lb.LB_ECFL),    # 2.334 * 0.05 / 0.1 > 1
    ((lb.LB_FD_D2Q16, 8, 8, 1e-3, 2e-3, 0.1, 3), lb.LB_ESTIFF),  # dt > tau
    ((lb.LB_CS_D2Q9 | lb.LB_IMEX, 8, 8, 0.8, 1.0, 1.0, 2), lb.LB_EINVAL),  # IMEX is FD only
    ((lb.LB_FD_D2Q16 | lb.LB_IMEX, 8, 8, 1e-3, 0.05, 0.1, 3), lb.LB_ECFL),  # IMEX keeps the CFL bound
    ((lb.LB_FD_D2Q16 | (1 << 11), 8, 8, 1e-3, 1e-4, 0.1, 3), lb.LB_EINVAL),  # unknown flag
    ((7, 8, 8, 0.8, 1.0, 1.0, 2), lb.LB_EINVAL),                # unknown model
    ((lb.LB_FD_D2Q9 | lb.LB_FP64, 32768, 16384, 1.0, 1e-5, 1e-4, 2), lb.LB_EINVAL),  # FD plane of 4 GiB
    ((lb.LB_FD_D2Q9, 32768, 32768, 1.0, 1e-5, 1e-4, 2), lb.LB_EINVAL),              # FD plane of 4 GiB
    ((lb.LB_FD_D2Q9 | lb.LB_FP16_SHIFTED, 32768, 32768, 1.0, 1e-5, 1e-4, 2), lb.LB_EINVAL),  # FP32 moment plane of 4 GiB
    # 896 bytes under 4 GiB unpadded, over it with the 4352-byte plane pad
    ((lb.LB_FD_D2Q9 | lb.LB_FP64, 536870800, 1, 1.0, 1e-5, 1e-4, 2), lb.LB_EINVAL),
    ((lb.LB_FD_D2Q16 | lb.LB_FP16_REF, 8, 8, 1e-3, 1e-4, 0.1, 3), lb.LB_EINVAL),  # reference-shifted FP16: CS only
    ((lb.LB_CS_D2Q9, 8, 8, float("nan"), 1.0, 1.0, 2), lb.LB_EINVAL),
])
def test_create_validation(args, code):
    h = lb._lib.lb_create(*args)
    assert not h
    assert lb.lb_last_error() == code
    assert lb.strerror(code) not in ("", "unknown status")


def test_tuning_cache_host_calls():
    # host-only entry points: no device needed
    assert lb._lib.lb_tuning_cache_clear() == lb.LB_OK
    assert lb.tuning_cache_size() == 0


def test_null_handles_are_rejected():
    assert lb._lib.lb_step(None, 1) == lb.LB_EINVAL
    assert lb._lib.lb_reduce(None, None) == lb.LB_EINVAL
    assert lb._lib.lb_steps_done(None) == -1
    lb._lib.lb_destroy(None)


def test_units_match_printed_values(golden):
    g = golden("tau_conversion.txt")
    for key in ("a", "b"):
        got = units.tau_lu_from_fd(float(g["shock_tau_fd_" + key]), int(g["shock_n"]))
        printed = g["shock_tau_lu_" + key]
        d = len(printed.split(".")[1])
        assert math.floor(got * 10 ** d + 1e-9) / 10 ** d == pytest.approx(float(printed), abs=1e-12)
    for n, printed in zip(g["table_n"].split(), g["table_tau_lu"].split()):
        got = units.tau_lu_from_fd(float(g["table_tau_fd"]), int(n))
        assert math.floor(got * 1e4 + 1e-9) / 1e4 == pytest.approx(float(printed), abs=1e-12)
        assert units.nu_cs(got, 1 / math.sqrt(3), 1.0) == pytest.approx(int(n) * float(g["table_tau_fd"]), rel=1e-12)
    t = golden("time_steps.txt")
    assert abs(units.cs_step_in_fd_time(int(t["n"])) - float(t["dt_cs_fd"])) < 5e-7
    # standard lattice units bridge
    assert units.tau_fd_from_std(0.6, 512) == pytest.approx(1.12764e-4, rel=1e-5)
    assert units.tau_std_from_lu(units.tau_lu_from_fd(units.tau_fd_from_std(0.8, 64), 64)) == pytest.approx(0.8)
    assert units.fd_time_step(5e-4, 1 / 2048, 3.324257, 0.5) == pytest.approx(7.3442e-5, rel=1e-4)


@pytest.mark.parametrize("kind,Nx,Ny", [("shear_y", 12, 7), ("shear_x", 12, 7), ("shear_x", 9, 1), ("tgv", 10, 6)])
def test_separable_patterns_match_the_initial_fields(kind, Nx, Ny):
    """The probe patterns of the diagnostics are the initial velocity
    patterns, as products of 1-D factors."""
    from paper_1904_02471_amd import workloads
    ax, ay, bx, by = workloads.separable_pattern(kind, Nx, Ny)
    assert ax.shape == bx.shape == (Nx,) and ay.shape == by.shape == (Ny,)
    if kind == "tgv":
        _, _, _, (px, py) = workloads.taylor_green(Nx, Ny, 1.0, 1.0)
    else:
        _, _, _, (px, py) = workloads.shear_wave(Nx, Ny, 1.0, kind[-1])
    np.testing.assert_allclose(np.outer(ay, ax), px, atol=1e-15)
    np.testing.assert_allclose(np.outer(by, bx), py, atol=1e-15)


def test_imex_lifts_the_stiffness_bound():
    """dt > tau passes validation with LB_IMEX (creation then proceeds to the
    device, which this host does not have, or succeeds on a GPU host)."""
    h = lb._lib.lb_create(lb.LB_FD_D2Q16 | lb.LB_IMEX, 8, 8, 1e-3, 2e-3, 0.1, 3)
    if h:
        lb._lib.lb_destroy(h)
    else:
        assert lb.lb_last_error() not in (lb.LB_ESTIFF, lb.LB_EINVAL, lb.LB_ECFL)


@pytest.mark.parametrize("omega", [0.0, 3.7])
def test_fit_decay_against_oracle_fit(omega):
    """lb_fit_decay (host FP64 least squares) against the oracle package's
    fit of the same series (numpy lstsq), on a decaying, modulated series."""
    from oracle import exact
    from paper_1904_02471_amd import serve
    t = np.linspace(0.0, 8.0, 401)
    amp = 0.01 * np.exp(-0.37 * t + 1e-3 * np.cos(3.7 * t + 0.4))  # ln|amp| exactly in the fitted form
    got = serve.fit_decay(t, amp, omega)
    want = exact.fit_decay_rate(t, amp) if omega == 0 else exact.fit_decay_rate_acoustic(t, amp, omega)
    assert got == pytest.approx(want, rel=1e-12, abs=1e-15)
    if omega:
        assert got == pytest.approx(0.37, rel=1e-12)
    else:
        assert got == pytest.approx(0.37, rel=1e-3)   # the modulation biases the plain fit
    with pytest.raises(lb.LBError):
        serve.fit_decay(t[:2], amp[:2])
    with pytest.raises(lb.LBError):
        serve.fit_decay(t, np.where(t > 4, 0.0, amp))
