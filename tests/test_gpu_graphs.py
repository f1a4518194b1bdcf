"""Graph replay of plain steps (lb_set_graph_steps): bitwise the same states
and diagnostics as launching every step, over several replays with eager
work and synchronisation between them, across lb_set_state (which drops the
captured graphs) and for odd graph lengths."""
import math

import numpy as np
import pytest

from paper_1904_02471_amd import lb, workloads

pytestmark = pytest.mark.gpu

CASES = [
    (lb.LB_CS_D2Q9, 64, 48, lb.LB_FP32),
    (lb.LB_CS_D2Q9, 37, 20, lb.LB_FP64),    # scalar row form
    (lb.LB_CS_D2Q9, 64, 16, lb.LB_FP16_SHIFTED),
    (lb.LB_FD_D2Q16, 70, 40, lb.LB_FP32),
    (lb.LB_FD_D2Q36, 33, 20, lb.LB_FP64),
]


def make(model, Nx, Ny, prec):
    if model == lb.LB_CS_D2Q9:
        return lb.Sim(model, Nx, Ny, 0.62, 1.0, 1.0, 2, precision=prec)
    ds = 1.0 / Nx
    vmax = lb.lb_model_info(model)[0].max()
    dt = 0.5 * ds / vmax
    return lb.Sim(model, Nx, Ny, 2 * dt, dt, ds, 4 if model == lb.LB_FD_D2Q36 else 3, precision=prec)


@pytest.mark.parametrize("model,Nx,Ny,prec", CASES)
def test_graph_replay_equals_step_by_step(model, Nx, Ny, prec):
    print("case: graphs", model, Nx, Ny, prec, flush=True)
    eager, graph = make(model, Nx, Ny, prec), make(model, Nx, Ny, prec)
    eager.set_graph_steps(0)
    f0 = workloads.random_distribution(eager.K, Nx, Ny, 5 + Nx, eager.w, spread=0.2)
    rho, ux, uy = workloads.random_state(Nx, Ny, 9 + Ny, eager.cs)
    for g in (eager, graph):
        g.set_state(f0)
        g.set_probe(*workloads.separable_pattern("tgv", Nx, Ny))
        g.series_reserve(64)
    # several replays, eager work (state reads) between them
    for n in (3, 21, 8, 1, 16):
        eager.step(n)
        graph.step(n)
        assert np.array_equal(eager.get_state(), graph.get_state()), n
    # runs between samples
    eager.step_sampled(37, 5)
    graph.step_sampled(37, 5)
    assert np.array_equal(eager.series_read(), graph.series_read())
    assert np.array_equal(eager.get_state(), graph.get_state())
    # a new state drops the graphs; an odd length is rounded up for CS
    for g in (eager, graph):
        g.init(rho, ux, uy)
    graph.set_graph_steps(3)
    for n in (7, 12, 5):
        eager.step(n)
        graph.step(n)
        assert np.array_equal(eager.get_state(), graph.get_state()), ("after init", n)
    assert eager.steps_done() == graph.steps_done() == 24


def test_graph_steps_argument_range():
    g = make(lb.LB_CS_D2Q9, 16, 8, lb.LB_FP32)
    with pytest.raises(lb.LBError):
        g.set_graph_steps(-2)
    with pytest.raises(lb.LBError):
        g.set_graph_steps(5000)
    g.set_graph_steps(-1)


@pytest.mark.parametrize("model,Nx,Ny,prec,shapes", [
    (lb.LB_CS_D2Q9, 256, 24, lb.LB_FP32, [(64, 8, 8), (256, 8, 8), (512, 8, 8), (1024, 8, 8)]),
    (lb.LB_CS_D2Q9, 100, 10, lb.LB_FP64, [(128, 8, 8)]),
    (lb.LB_FD_D2Q16, 70, 40, lb.LB_FP32, [(0, 4, 4), (0, 8, 4), (0, 4, 8)]),
    (lb.LB_FD_D2Q36, 65, 33, lb.LB_FP64, [(0, 4, 4), (0, 8, 4)]),
    (lb.LB_FD_D2Q36, 70, 37, lb.LB_FP32, [(0, 4, 4), (0, 8, 4)]),
    (lb.LB_FD_D2Q16, 64, 48, lb.LB_FP16_SHIFTED, [(0, 4, 4), (0, 8, 4)]),
])
def test_launch_shapes_do_not_change_results(model, Nx, Ny, prec, shapes):
    """Every tuned launch shape (CS workgroup size, FD tile height) gives
    bitwise the same states and diagnostics; autotuning leaves the state
    untouched and picks one of the candidates."""
    print("case: tuning", model, Nx, Ny, prec, flush=True)
    f0 = None
    ref = None
    for shape in [None] + shapes:
        g = make(model, Nx, Ny, prec)
        if f0 is None:
            f0 = workloads.random_distribution(g.K, Nx, Ny, 3 + Nx, g.w, spread=0.2)
        g.set_state(f0)
        g.set_probe(*workloads.separable_pattern("tgv", Nx, Ny))
        g.series_reserve(16)
        if shape is not None:
            g.set_tuning(*shape)
            assert g.tuning() == shape
        g.step(9)
        g.step_sampled(23, 4)
        out = (g.get_state(), g.series_read())
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]), shape
            assert np.array_equal(out[1], ref[1]), shape
    g = make(model, Nx, Ny, prec)
    g.set_state(f0)
    g.set_probe(*workloads.separable_pattern("tgv", Nx, Ny))
    g.series_reserve(16)
    before = g.get_state()
    cs_threads, fd_rows, fd_rows_rest = g.autotune(3)
    assert np.array_equal(g.get_state(), before)
    assert fd_rows in (4, 8) and fd_rows_rest in (4, 8) and cs_threads in (0, 256, 512, 1024)
    g.step(9)
    g.step_sampled(23, 4)
    assert np.array_equal(g.get_state(), ref[0])
    assert np.array_equal(g.series_read(), ref[1])


def test_autotune_cache():
    """lb_autotune keeps its choice per device, model, storage, boundaries,
    grid and order: a second handle of the same key takes the cached shapes
    (whatever shapes it held) without a new entry, a new grid or model adds
    one, and clearing the cache empties it."""
    print("case: autotune cache", flush=True)
    lb.tuning_cache_clear()
    assert lb.tuning_cache_size() == 0
    sims = []
    for Nx, Ny in ((96, 80), (96, 80), (128, 80)):
        g = make(lb.LB_FD_D2Q16, Nx, Ny, lb.LB_FP32)
        rho, ux, uy = workloads.random_state(Nx, Ny, 5, 1.0)
        g.init(rho, ux, uy)
        sims.append(g)
    first = sims[0].autotune(2), sims[0].fd_fused()
    assert lb.tuning_cache_size() == 1
    other = (0, 4, 8) if first[0] != (0, 4, 8) else (0, 8, 4)
    sims[1].set_tuning(*other)
    sims[1].set_fd_fused(0 if first[1] else 32)
    assert (sims[1].autotune(2), sims[1].fd_fused()) == first
    assert lb.tuning_cache_size() == 1
    sims[2].autotune(2)
    assert lb.tuning_cache_size() == 2
    cs = make(lb.LB_CS_D2Q9, 96, 80, lb.LB_FP32)
    rho, ux, uy = workloads.random_state(96, 80, 6, 3.0 ** -0.5)
    cs.init(rho, ux, uy)
    cs.autotune(2)
    assert lb.tuning_cache_size() == 3
    lb.tuning_cache_clear()
    assert lb.tuning_cache_size() == 0


@pytest.mark.parametrize("prec,Nx,Ny", [(lb.LB_FP32, 128, 40), (lb.LB_FP16_SHIFTED, 96, 24),
                                        (lb.LB_FP16_REF, 64, 20), (lb.LB_FP64, 68, 12)])
def test_cs_store_policy_does_not_change_results(prec, Nx, Ny):
    """Non-temporal stores of the CS vector rows give bitwise the states and
    diagnostics of plain stores, with graph replay and sampled steps mixed
    in; the policy is rejected for FD handles."""
    print("case: CS store policy", prec, Nx, Ny, flush=True)
    out = []
    for nt in (False, True):
        g = make(lb.LB_CS_D2Q9, Nx, Ny, prec)
        rho, ux, uy = workloads.random_state(Nx, Ny, 11, 3.0 ** -0.5)
        g.init(rho, ux, uy)
        g.set_probe(*workloads.separable_pattern("tgv", Nx, Ny))
        g.series_reserve(16)
        g.set_cs_nontemporal(nt)
        assert g.cs_nontemporal() == nt
        g.step(19)
        g.step_sampled(21, 4)
        g.step(3)
        out.append((g.get_state(), g.series_read()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    fd = make(lb.LB_FD_D2Q16, 16, 16, lb.LB_FP32)
    with pytest.raises(lb.LBError):
        fd.set_cs_nontemporal(True)
