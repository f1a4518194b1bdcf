"""The temporally blocked FD step (lb_set_fd_fused: the three Runge-Kutta
stages in one launch, stage values kept on chip) against the three stage
launches, bit for bit, and against the FP64 oracle: strips and segments
with ragged tails, grids narrower than one strip or one segment, several
steps, graph replay, the 2048^2 workload."""
import math

import numpy as np
import pytest

from paper_1904_02471_amd import lb, workloads
from tests.gpu_helpers import assert_state_close, pair, tolerance

pytestmark = pytest.mark.gpu

VMAX = {lb.LB_FD_D2Q9: math.sqrt(3), lb.LB_FD_D2Q16: 2.3344142183389773}


def fd_args(model, n):
    ds = 1.0 / n
    dt = 0.5 * ds / VMAX[model]
    return 2.0 * dt, dt, ds


def twin(model, Nx, Ny, N, ys, seed=3):
    """Two FP32 simulations of one random state: stage launches and fused."""
    tau, dt, ds = fd_args(model, max(Nx, Ny))
    a = lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=lb.LB_FP32)
    b = lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=lb.LB_FP32)
    rho, ux, uy = workloads.random_state(Nx, Ny, seed, 1.0, u_max=0.08)
    for s in (a, b):
        s.set_graph_steps(0)
        s.init(rho, ux, uy)
    b.set_fd_fused(ys)
    return a, b


@pytest.mark.parametrize("model,N", [(lb.LB_FD_D2Q16, 3), (lb.LB_FD_D2Q16, 1), (lb.LB_FD_D2Q9, 2)])
@pytest.mark.parametrize("shape,ys", [((8, 8), 64), ((70, 45), 16), ((130, 17), 8), ((111, 40), 32),
                                      ((1, 9), 4), ((9, 1), 2), ((3, 2), 64), ((257, 130), 48)])
def test_fused_equals_stage_launches(model, N, shape, ys):
    Nx, Ny = shape
    print("case: fused vs stages", model, N, shape, ys, flush=True)
    a, b = twin(model, Nx, Ny, N, ys)
    done = 0
    for n in (1, 3, 8):
        a.step(n - done)
        b.step(n - done)
        done = n
        fa, fb = a.get_state(), b.get_state()
        bad = np.argwhere(fa != fb)
        assert bad.size == 0, "fused differs after %d steps at %s (of %d)" % (n, bad[:5].tolist(), len(bad))
        ra, rb = a.moments(), b.moments()
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y)


def test_fused_against_oracle():
    """A 70 x 45 D2Q16 state, fused steps against the FP64 oracle."""
    print("case: fused vs oracle", flush=True)
    Nx, Ny = 70, 45
    tau, dt, ds = fd_args(lb.LB_FD_D2Q16, Nx)
    g, o = pair(lb.LB_FD_D2Q16, Nx, Ny, tau, dt, ds, 3, lb.LB_FP32)
    g.set_fd_fused(32)
    rho, ux, uy = workloads.random_state(Nx, Ny, 8, 1.0, u_max=0.1)
    g.init(rho, ux, uy)
    o.init(rho, ux, uy)
    for n in (1, 4):
        g.step(1 if n == 1 else 3)
        o.step(1 if n == 1 else 3)
        fo = o.get_state()
        assert_state_close(g.get_state(), fo, tolerance(lb.LB_FP32, n, fo, g.w, fo.sum(0).mean()),
                           "fused 70x45 after %d steps" % n)


def test_fused_graph_replay_and_sampled_steps():
    """Graph replay (odd graph lengths round up to keep the buffer pair in
    place) and sampled steps (stage launches with the diagnostics) mixed with
    fused plain steps: the same states and series as the stage launches."""
    print("case: fused graphs and sampling", flush=True)
    a, b = twin(lb.LB_FD_D2Q16, 96, 80, 3, 32, seed=5)
    for s in (a, b):
        s.set_graph_steps(3)
        s.series_reserve(64)
        s.set_probe(*workloads.separable_pattern("tgv", 96, 80))
    a.step_sampled(23, 5)
    b.step_sampled(23, 5)
    a.step(7)
    b.step(7)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.series_read(), b.series_read())


def test_fused_2048_workload():
    """The 2048^2 D2Q16 vortex of the benchmark, autotuned launch shapes,
    two steps: bitwise the stage launches' state."""
    print("case: fused 2048", flush=True)
    from paper_1904_02471_amd import units
    n = 2048
    ds = 1.0 / n
    tau = units.tau_fd_from_std(0.6, n)
    dt = units.fd_time_step(tau, ds, VMAX[lb.LB_FD_D2Q16], 0.5)
    rho, ux, uy, _ = workloads.taylor_green(n, n, units.velocity_fd_from_std(0.01), 1.0)
    out = []
    for ys in (0, 64):
        g = lb.Sim(lb.LB_FD_D2Q16, n, n, tau, dt, ds, 3, precision=lb.LB_FP32)
        g.init(rho, ux, uy)
        g.set_fd_fused(ys)
        g.step(2)
        out.append(g.moments())
        if ys:
            f_fused = g.get_state()
        else:
            f_stage = g.get_state()
        g.destroy()
    assert np.array_equal(f_fused, f_stage)
    for x, y in zip(*out):
        assert np.array_equal(x, y)


def test_fused_rejections_and_tuning():
    tau, dt, ds = fd_args(lb.LB_FD_D2Q16, 16)
    for prec in (lb.LB_FP64, lb.LB_FP16_SHIFTED):
        g = lb.Sim(lb.LB_FD_D2Q16, 16, 16, tau, dt, ds, 3, precision=prec)
        with pytest.raises(lb.LBError):
            g.set_fd_fused(32)
    g = lb.Sim(lb.LB_FD_D2Q36, 16, 16, 1e-2, 0.4 / 16 / 3.33, 1.0 / 16, 4)
    with pytest.raises(lb.LBError):
        g.set_fd_fused(32)
    g = lb.Sim(lb.LB_CS_D2Q9, 16, 16, 0.7, 1.0, 1.0, 2)
    with pytest.raises(lb.LBError):
        g.set_fd_fused(32)
    g = lb.Sim(lb.LB_FD_D2Q16, 16, 16, tau, dt, ds, 3)
    g.set_bc_x(1.1, 0.9)
    with pytest.raises(lb.LBError):
        g.set_fd_fused(32)
    g = lb.Sim(lb.LB_FD_D2Q16, 256, 256, tau, dt, ds, 3)
    rho, ux, uy = workloads.random_state(256, 256, 2, 1.0)
    g.init(rho, ux, uy)
    g.autotune(2)
    assert g.fd_fused() in (0, 32, 64, 128)
