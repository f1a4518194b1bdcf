"""GPU parity: the HIP path through the C ABI against the FP64 oracle,
element by element, on seeded inputs (brute force on small lattices, several
tiles with ragged tails, fixed ends, every precision)."""
import math

import numpy as np
import pytest

from paper_1904_02471_amd import lb, workloads
from tests.gpu_helpers import PREC_NAME, U16, assert_state_close, field_errors, pair, tolerance

pytestmark = pytest.mark.gpu

PRECS = [lb.LB_FP64, lb.LB_FP32, lb.LB_FP16_SHIFTED]
CS_PRECS = PRECS + [lb.LB_FP16_REF]   # FP16 relative to a reference equilibrium: CS only


def cs_case(Nx, Ny, tau=0.7, prec=lb.LB_FP32, bc=None, dsdt=(1.0, 1.0)):
    return pair(lb.LB_CS_D2Q9, Nx, Ny, tau, dsdt[1], dsdt[0], 2, prec, bc=bc)


def fd_params(model, Nx):
    ds = 1.0 / Nx
    vmax = {lb.LB_FD_D2Q9: math.sqrt(3), lb.LB_FD_D2Q16: 2.3344142183389773,
            lb.LB_FD_D2Q25: 2.8569700138728056, lb.LB_FD_D2Q36: 3.3242574335521193}[model]
    dt = 0.5 * ds / vmax
    return ds, dt, 2.0 * dt


def run_and_compare(g, o, steps, prec, what, fields=False):
    """Step both sides and compare the states element by element after each
    count in `steps`; with `fields` (FP32), also rho - rho0 and u against the
    oracle's within 1e-5 relative L2 after up to 10 steps (later, a random
    initial state has relaxed toward uniform density and |rho - rho0|
    shrinks by orders of magnitude, so the relative figure no longer
    measures the scheme; the element-wise bound still holds)."""
    done = 0
    for n in steps:
        g.step(n - done)
        o.step(n - done)
        done = n
        fo = o.get_state()
        fg = g.get_state()
        rho0 = fo.sum(0).mean()
        tol = tolerance(prec, n, fo, g.w, rho0)
        assert_state_close(fg, fo, tol, "%s after %d steps" % (what, n))
        if prec in (lb.LB_FP16_SHIFTED, lb.LB_FP16_REF):
            # stochastic rounding: unbiased errors of at most one FP16 step
            # (2 u16 |g|) per rounding, variance at most a quarter step squared;
            # over the initial and n stepped roundings without amplification
            # the rms error is at most u16 sqrt(n+1) rms g.  Asserted with a
            # factor 2 (measured: 0.15-0.83 over these cases)
            go = fo - g.w[:, None, None] * rho0
            ratio = np.sqrt(np.mean((fg - fo) ** 2)) / (U16 * np.sqrt(n + 1) * np.sqrt(np.mean(go ** 2)))
            print("%s after %d steps: rms error / (u16 sqrt(n+1) rms g) = %.3f" % (what, n, ratio), flush=True)
            assert ratio <= 2.0, (what, n, ratio)
        if fields:
            e_rho, e_u = field_errors(g, o)
            print("%s after %d steps: rel-L2 rho-rho0 %.2e u %.2e" % (what, n, e_rho, e_u), flush=True)
            if n <= 10:
                assert e_rho <= 1e-5 and e_u <= 1e-5


@pytest.mark.parametrize("prec", CS_PRECS, ids=lambda p: PREC_NAME[p])
def test_cs_8x8_random_state(prec):
    print("case: cs 8x8 random non-equilibrium state", PREC_NAME[prec], flush=True)
    g, o = cs_case(8, 8, prec=prec)
    f0 = workloads.random_distribution(9, 8, 8, 1904, g.w, spread=0.3)
    g.set_state(f0)
    o.set_state(f0)
    # the state transfer itself is exact up to the storage rounding
    assert_state_close(g.get_state(), f0, tolerance(prec, 0, f0, g.w, f0.sum(0).mean()), "cs set/get state")
    run_and_compare(g, o, [1, 10, 100], prec, "cs 8x8 " + PREC_NAME[prec], fields=prec == lb.LB_FP32)


@pytest.mark.parametrize("shape", [(37, 23), (300, 5), (1, 7), (5, 1), (257, 130)])
def test_cs_ragged_shapes(shape):
    Nx, Ny = shape
    print("case: cs ragged", shape, flush=True)
    g, o = cs_case(Nx, Ny, tau=0.6)
    rho, ux, uy = workloads.random_state(Nx, Ny, 7 + Nx, g.cs)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 5, 20], lb.LB_FP32, "cs %dx%d" % shape)


@pytest.mark.parametrize("prec", CS_PRECS, ids=lambda p: PREC_NAME[p])
@pytest.mark.parametrize("Nx", [4, 8, 12, 260, 516, 2052, 4100])
def test_cs_vector_rows(Nx, prec):
    """Periodic rows whose width is a multiple of the chunk width take the
    vector row form: one chunk, a partial wave, the edge lanes of several
    waves and several chunks per thread (rows wider than 1024 chunks)."""
    print("case: cs vector rows", Nx, PREC_NAME[prec], flush=True)
    Ny = 3
    g, o = cs_case(Nx, Ny, tau=0.65, prec=prec)
    f0 = workloads.random_distribution(9, Nx, Ny, 11 + Nx, g.w, spread=0.2)
    g.set_state(f0)
    o.set_state(f0)
    run_and_compare(g, o, [1, 4], prec, "cs vector rows %d %s" % (Nx, PREC_NAME[prec]))


@pytest.mark.parametrize("shape", [(37, 23), (1, 7), (5, 1), (6, 3)])
def test_cs_fp16_ref_scalar_rows(shape):
    """FP16 relative to a reference equilibrium on rows the vector form does
    not take (widths not a multiple of 4): the scalar row form, from an
    initial equilibrium and then from a set non-equilibrium state; the
    reference follows each (velocity of the initial fields, of the set
    state)."""
    Nx, Ny = shape
    print("case: cs fp16ref scalar rows", shape, flush=True)
    g, o = cs_case(Nx, Ny, tau=0.6, prec=lb.LB_FP16_REF)
    rho, ux, uy = workloads.random_state(Nx, Ny, 9 + Nx, g.cs)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 5, 20], lb.LB_FP16_REF, "cs fp16ref %dx%d" % shape)
    f0 = workloads.random_distribution(9, Nx, Ny, 5 + Ny, g.w, spread=0.2)
    g.set_state(f0)
    o.set_state(f0)
    assert_state_close(g.get_state(), f0, tolerance(lb.LB_FP16_REF, 0, f0, g.w, f0.sum(0).mean()),
                       "cs fp16ref set/get state")
    run_and_compare(g, o, [1, 7], lb.LB_FP16_REF, "cs fp16ref state %dx%d" % shape)


def test_cs_fp16_ref_rejections():
    """Reference-shifted FP16 storage: collision-streaming and periodic only."""
    g = lb.Sim(lb.LB_CS_D2Q9, 8, 8, 0.7, 1.0, 1.0, 2, precision=lb.LB_FP16_REF)
    with pytest.raises(lb.LBError) as e:
        g.set_bc_x(1.1, 0.9)
    assert e.value.code == lb.LB_EINVAL
    with pytest.raises(lb.LBError) as e:
        lb.Sim(lb.LB_FD_D2Q16, 8, 8, 1e-2, 1e-3, 0.1, 3, precision=lb.LB_FP16_REF)
    assert e.value.code == lb.LB_EINVAL


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_NAME[p])
def test_cs_fixed_ends(prec):
    print("case: cs fixed ends 19x6", PREC_NAME[prec], flush=True)
    g, o = cs_case(19, 6, tau=0.8, prec=prec, bc=(1.3, 0.8))
    f0 = workloads.random_distribution(9, 19, 6, 33, g.w, spread=0.3)
    g.set_state(f0)
    o.set_state(f0)
    run_and_compare(g, o, [1, 2, 30], prec, "cs fixed " + PREC_NAME[prec])


def test_cs_paper_units():
    # ds = 1, dt = 1/sqrt(3): c_s = 1, the paper's CS convention
    print("case: cs paper units", flush=True)
    g, o = cs_case(16, 12, tau=0.35, dsdt=(1.0, 1.0 / math.sqrt(3)), prec=lb.LB_FP64)
    rho, ux, uy = workloads.random_state(16, 12, 5, g.cs)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 25], lb.LB_FP64, "cs paper units")


FD_MODELS = [(lb.LB_FD_D2Q9, 2), (lb.LB_FD_D2Q16, 3), (lb.LB_FD_D2Q25, 4), (lb.LB_FD_D2Q36, 4),
             (lb.LB_FD_D2Q16, 1), (lb.LB_FD_D2Q36, 5)]


@pytest.mark.parametrize("model,N", FD_MODELS)
@pytest.mark.parametrize("prec", [lb.LB_FP64, lb.LB_FP32], ids=lambda p: PREC_NAME[p])
def test_fd_8x8_random_state(model, N, prec):
    print("case: fd 8x8 model", model, "N", N, PREC_NAME[prec], flush=True)
    ds, dt, tau = fd_params(model, 8)
    g, o = pair(model, 8, 8, tau, dt, ds, N, prec)
    f0 = workloads.random_distribution(g.K, 8, 8, 11 + model, g.w, spread=0.3)
    g.set_state(f0)
    o.set_state(f0)
    run_and_compare(g, o, [1, 3, 10], prec, "fd model %d N %d %s" % (model, N, PREC_NAME[prec]),
                    fields=prec == lb.LB_FP32)


@pytest.mark.parametrize("model,N", [(lb.LB_FD_D2Q16, 3), (lb.LB_FD_D2Q36, 4), (lb.LB_FD_D2Q9, 2)])
def test_fd_ragged_tiles(model, N):
    # 70 x 45: two tiles in x (tail 6) and three in y (tail 13)
    Nx, Ny = 70, 45
    print("case: fd ragged", Nx, Ny, model, flush=True)
    ds, dt, tau = fd_params(model, Nx)
    g, o = pair(model, Nx, Ny, tau, dt, ds, N, lb.LB_FP32)
    rho, ux, uy = workloads.random_state(Nx, Ny, 3, 1.0, u_max=0.1)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 4], lb.LB_FP32, "fd %dx%d" % (Nx, Ny), fields=True)


@pytest.mark.parametrize("shape", [(1, 9), (9, 1), (3, 2), (130, 17)])
def test_fd_degenerate_shapes(shape):
    Nx, Ny = shape
    print("case: fd degenerate", shape, flush=True)
    ds, dt, tau = fd_params(lb.LB_FD_D2Q16, max(Nx, Ny))
    g, o = pair(lb.LB_FD_D2Q16, Nx, Ny, tau, dt, ds, 3, lb.LB_FP64)
    rho, ux, uy = workloads.random_state(Nx, Ny, 2, 1.0)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 3], lb.LB_FP64, "fd %dx%d" % shape)


@pytest.mark.parametrize("prec", [lb.LB_FP64, lb.LB_FP32, lb.LB_FP16_SHIFTED], ids=lambda p: PREC_NAME[p])
def test_fd_fixed_ends(prec):
    Nx, Ny = 70, 5
    print("case: fd fixed ends", PREC_NAME[prec], flush=True)
    ds, dt, tau = fd_params(lb.LB_FD_D2Q36, Nx)
    g, o = pair(lb.LB_FD_D2Q36, Nx, Ny, tau, dt, ds, 4, prec, bc=(1.5, 1.0))
    rho, ux, uy = workloads.shock_tube(Nx, Ny, 1.5, 1.0, width=2.0)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    run_and_compare(g, o, [1, 10], prec, "fd fixed " + PREC_NAME[prec])


@pytest.mark.parametrize("eps", [1e30, 1e-6, 1e-12])
def test_fd_weno_eps(eps):
    print("case: fd weno eps", eps, flush=True)
    ds, dt, tau = fd_params(lb.LB_FD_D2Q16, 16)
    g, o = pair(lb.LB_FD_D2Q16, 16, 12, tau, dt, ds, 3, lb.LB_FP64, eps=eps)
    f0 = workloads.random_distribution(16, 16, 12, 4, g.w, spread=0.3)
    g.set_state(f0)
    o.set_state(f0)
    run_and_compare(g, o, [1, 5], lb.LB_FP64, "fd eps %g" % eps)


@pytest.mark.parametrize("model", [lb.LB_CS_D2Q9, lb.LB_FD_D2Q16])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_NAME[p])
def test_moments_and_reduce(model, prec):
    Nx, Ny = 40, 24
    print("case: moments/reduce", model, PREC_NAME[prec], flush=True)
    if model == lb.LB_CS_D2Q9:
        g, o = cs_case(Nx, Ny, tau=0.6, prec=prec)
    else:
        ds, dt, tau = fd_params(model, Nx)
        g, o = pair(model, Nx, Ny, tau, dt, ds, 3, prec)
    rho, ux, uy, _ = workloads.taylor_green(Nx, Ny, 0.05 * g.cs, g.cs ** 2)
    ax, ay, bx, by = workloads.separable_pattern("tgv", Nx, Ny)
    px, py = np.outer(ay, ax), np.outer(by, bx)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    g.set_probe(ax, ay, bx, by)
    g.step(7)
    o.step(7)
    rg, xg, yg = g.moments()
    ro, xo, yo = o.moments()
    scale = 0.05 * g.cs
    tol = {lb.LB_FP64: 1e-12, lb.LB_FP32: 1e-6, lb.LB_FP16_SHIFTED: 2e-3}[prec]
    assert np.max(np.abs(rg - ro)) <= tol
    assert np.max(np.abs(xg - xo)) <= tol * scale * 10 + tol * 1e-2
    assert np.max(np.abs(yg - yo)) <= tol * scale * 10 + tol * 1e-2
    dg = g.reduce()
    do = o.reduce(px, py)
    print("reduce gpu", dg, "oracle", do, flush=True)
    assert dg[0] == pytest.approx(do[0], rel=max(tol, 1e-13))
    for i in (1, 2):
        assert abs(dg[i] - do[i]) <= tol * do[0] * scale
    assert dg[3] == pytest.approx(do[3], rel=max(10 * tol, 1e-11))
    assert dg[4] == pytest.approx(do[4], rel=max(10 * tol, 1e-11))


@pytest.mark.parametrize("model", [lb.LB_CS_D2Q9, lb.LB_FD_D2Q16])
def test_run_sampled_matches_stepwise(model):
    Nx, Ny = 64, 48
    print("case: run_sampled", model, flush=True)
    if model == lb.LB_CS_D2Q9:
        g, o = cs_case(Nx, Ny, tau=0.6, prec=lb.LB_FP64)
    else:
        ds, dt, tau = fd_params(model, Nx)
        g, o = pair(model, Nx, Ny, tau, dt, ds, 3, lb.LB_FP64)
    rho, ux, uy, _ = workloads.taylor_green(Nx, Ny, 0.02 * g.cs, g.cs ** 2)
    ax, ay, bx, by = workloads.separable_pattern("tgv", Nx, Ny)
    px, py = np.outer(ay, ax), np.outer(by, bx)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    g.set_probe(ax, ay, bx, by)
    series = g.run_sampled(30, 10)
    assert series.shape == (4, 5)
    for i in range(4):
        if i:
            o.step(10)
        want = o.reduce(px, py)
        np.testing.assert_allclose(series[i], want, rtol=1e-11, atol=1e-14 * abs(want[0]))
    assert g.steps_done() == 30


def test_state_roundtrip_and_restart():
    # stepping n then m equals n + m; save / restore continues bitwise
    print("case: restart", flush=True)
    for model in (lb.LB_CS_D2Q9, lb.LB_FD_D2Q16):
        if model == lb.LB_CS_D2Q9:
            a = lb.Sim(model, 33, 20, 0.7, 1.0, 1.0, 2, precision=lb.LB_FP64)
            b = lb.Sim(model, 33, 20, 0.7, 1.0, 1.0, 2, precision=lb.LB_FP64)
        else:
            ds, dt, tau = fd_params(model, 33)
            a = lb.Sim(model, 33, 20, tau, dt, ds, 3, precision=lb.LB_FP64)
            b = lb.Sim(model, 33, 20, tau, dt, ds, 3, precision=lb.LB_FP64)
        rho, ux, uy = workloads.random_state(33, 20, 9, a.cs)
        a.init(rho, ux, uy)
        b.init(rho, ux, uy)
        a.step(5)
        a.step(7)
        b.step(12)
        assert np.array_equal(a.get_state(), b.get_state())
        f = a.get_state()
        c = lb.Sim(a.model, 33, 20, a.tau, a.dt, a.ds, a.N, precision=lb.LB_FP64)
        c.set_state(f)
        c.step(3)
        a.step(3)
        np.testing.assert_allclose(c.get_state(), a.get_state(), rtol=0, atol=1e-14)


def test_uniform_state_stays_uniform_and_rest_is_exact():
    print("case: uniform", flush=True)
    for prec in PRECS:
        g = lb.Sim(lb.LB_CS_D2Q9, 40, 30, 0.7, 1.0, 1.0, 2, precision=prec)
        g.init(np.full((30, 40), 1.03), np.full((30, 40), 0.02), np.full((30, 40), -0.01))
        g.step(20)
        f = g.get_state()
        # stochastic rounding (FP16): uniform in distribution, every value
        # within a few FP16 ulps of the largest stored (shifted) magnitude
        gmax = max(abs(f[k].mean() - g.w[k] * 1.03) for k in range(9))  # rho0 = 1.03
        for k in range(9):
            if prec == lb.LB_FP16_SHIFTED:
                assert np.abs(f[k] - f[k].mean()).max() <= 8 * 2.0 ** -11 * gmax
            else:
                assert np.all(f[k] == f[k, 0, 0])
        # rho = rho0, u = 0: the shifted state is exactly zero and stays so
        g.init(np.ones((30, 40)), np.zeros((30, 40)), np.zeros((30, 40)))
        g.step(10)
        assert np.array_equal(g.get_state(), np.broadcast_to(g.w[:, None, None], (9, 30, 40)))
        ds, dt, tau = fd_params(lb.LB_FD_D2Q16, 70)
        if prec != lb.LB_FP16_SHIFTED:
            h = lb.Sim(lb.LB_FD_D2Q16, 70, 20, tau, dt, ds, 3, precision=prec)
            h.init(np.full((20, 70), 1.02), np.full((20, 70), 0.03), np.full((20, 70), -0.02))
            h.step(3)
            f = h.get_state()
            for k in range(16):
                assert np.all(f[k] == f[k, 0, 0])


def test_error_paths():
    g = lb.Sim(lb.LB_CS_D2Q9, 8, 8, 0.7, 1.0, 1.0, 2)
    with pytest.raises(lb.LBError) as e:
        g.step(1)                                  # before init
    assert e.value.code == lb.LB_ESTATE
    with pytest.raises(lb.LBError) as e:
        g.init(np.full((8, 8), -1.0), np.zeros((8, 8)), np.zeros((8, 8)))
    assert e.value.code == lb.LB_EINVAL
    g.init(np.ones((8, 8)), np.zeros((8, 8)), np.zeros((8, 8)))
    with pytest.raises(lb.LBError) as e:
        g.set_bc_x(1.0, 1.0)                       # after init
    assert e.value.code == lb.LB_ESTATE
    with pytest.raises(lb.LBError):
        g.set_weno_eps(1e-6)                       # CS has no WENO
    with pytest.raises(lb.LBError):
        g.run_sampled(10, 0)
    assert g.device_bytes() >= 2 * 9 * 64 * 4


def test_step_sampled_series():
    print("case: step_sampled series", flush=True)
    g = lb.Sim(lb.LB_CS_D2Q9, 48, 32, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP64)
    o = lb.Sim(lb.LB_CS_D2Q9, 48, 32, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP64)
    rho, ux, uy, _ = workloads.taylor_green(48, 32, 0.02, 1.0 / 3.0)
    ax, ay, bx, by = workloads.separable_pattern("tgv", 48, 32)
    for s in (g, o):
        s.init(rho, ux, uy)
        s.set_probe(ax, ay, bx, by)
    with pytest.raises(lb.LBError) as e:
        g.step_sampled(5, 5)               # no capacity reserved
    assert e.value.code == lb.LB_EBUSY
    g.series_reserve(8)
    g.step_sampled(7, 5)                   # samples t = 0, 5
    g.step_sampled(6, 5)                   # samples t = 10
    rows = g.series_read()
    assert [int(t) for t in rows[:, 0]] == [0, 5, 10]
    ref = o.run_sampled(10, 5)
    np.testing.assert_allclose(rows[:, 1:], ref, rtol=1e-12, atol=1e-15 * ref[0, 0])
    assert g.series_read().shape == (0, 6)


@pytest.mark.parametrize("model", [lb.LB_CS_D2Q9, lb.LB_FD_D2Q16])
@pytest.mark.parametrize("prec", [lb.LB_FP64, lb.LB_FP32], ids=lambda p: PREC_NAME[p])
def test_reduce_field(model, prec):
    """lb_reduce_field: diagnostics with an arbitrary (non-separable) velocity
    pattern against the oracle's, and with a separable one against lb_reduce
    (same sums in the same order: M, P, E bitwise, A to rounding)."""
    Nx, Ny = 70, 45
    print("case: reduce_field", model, PREC_NAME[prec], flush=True)
    if model == lb.LB_CS_D2Q9:
        g, o = cs_case(Nx, Ny, tau=0.6, prec=prec)
    else:
        ds, dt, tau = fd_params(model, Nx)
        g, o = pair(model, Nx, Ny, tau, dt, ds, 3, prec)
    rho, ux, uy = workloads.random_state(Nx, Ny, 41, g.cs, u_max=0.05)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    g.step(3)
    o.step(3)
    rng = np.random.default_rng(1905)
    px, py = rng.standard_normal((Ny, Nx)), rng.standard_normal((Ny, Nx))
    dg = g.reduce_field(px, py)
    do = o.reduce(px, py)
    tol = 1e-12 if prec == lb.LB_FP64 else 1e-6
    print("reduce_field gpu", dg, "oracle", do, flush=True)
    assert dg[0] == pytest.approx(do[0], rel=max(tol, 1e-13))
    for i in (1, 2):
        assert abs(dg[i] - do[i]) <= tol * do[0] * 0.05 * g.cs
    assert dg[3] == pytest.approx(do[3], rel=10 * tol)
    _, xo, yo = o.moments()
    a_scale = float(np.sum(np.abs(xo * px) + np.abs(yo * py)) / np.sum(px * px + py * py))
    assert abs(dg[4] - do[4]) <= 10 * tol * a_scale
    # no pattern: A = 0, the rest unchanged
    d0 = g.reduce_field()
    assert d0[4] == 0.0 and np.array_equal(d0[:4], dg[:4])
    # a separable pattern through both entry points
    ax, ay, bx, by = workloads.separable_pattern("tgv", Nx, Ny)
    g.set_probe(ax, ay, bx, by)
    dr = g.reduce()
    df = g.reduce_field(np.outer(ay, ax), np.outer(by, bx))
    assert np.array_equal(dr[:4], df[:4])
    assert df[4] == pytest.approx(dr[4], rel=1e-12)
