"""GPU parity at the benchmark's full size (2048 x 2048 Taylor-Green vortex,
FP32, the launch configuration bench.py times), on sampled nodes: the oracle
recomputes each sampled node on a periodic window around it that is wider
than the stencil reach of the steps taken, so the window's wrap-around never
reaches the sampled node.  Plus properties that hold at any size
(conservation, determinism, sampled diagnostics)."""
import numpy as np
import pytest

import oracle
from paper_1904_02471_amd import lb, units, workloads
from tests.gpu_helpers import ORACLE_MODEL, tolerance

pytestmark = pytest.mark.gpu

N = 2048


def bench_cs():
    g = lb.Sim(lb.LB_CS_D2Q9, N, N, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP32)
    r, ux, uy, _ = workloads.taylor_green(N, N, 0.01, 1.0 / 3.0)
    g.init(r, ux, uy)
    return g, (r, ux, uy), dict(tau=0.6, dt=1.0, ds=1.0, N=2), 1


def bench_fd():
    ds = 1.0 / N
    tau = units.tau_fd_from_std(0.6, N)
    dt = units.fd_time_step(tau, ds, lb.lb_model_info(lb.LB_FD_D2Q16)[0].max(), 0.5)
    g = lb.Sim(lb.LB_FD_D2Q16, N, N, tau, dt, ds, 3, precision=lb.LB_FP32)
    r, ux, uy, _ = workloads.taylor_green(N, N, units.velocity_fd_from_std(0.01), 1.0)
    g.init(r, ux, uy)
    return g, (r, ux, uy), dict(tau=tau, dt=dt, ds=ds, N=3), 9   # reach: 3 stages x 3 nodes


def tgv4096_cs(prec):
    n = 4096
    g = lb.Sim(lb.LB_CS_D2Q9, n, n, 0.55, 1.0, 1.0, 2, precision=prec)
    r, ux, uy, _ = workloads.taylor_green(n, n, 0.01, 1.0 / 3.0)
    g.init(r, ux, uy)
    return g, (r, ux, uy), dict(tau=0.55, dt=1.0, ds=1.0, N=2), 1


def tgv2048_fd36():
    ds = 1.0 / N
    tau = 5e-4
    dt = units.fd_time_step(tau, ds, lb.lb_model_info(lb.LB_FD_D2Q36)[0].max(), 0.5)
    g = lb.Sim(lb.LB_FD_D2Q36, N, N, tau, dt, ds, 4, precision=lb.LB_FP32)
    r, ux, uy, _ = workloads.taylor_green(N, N, 0.01, 1.0)
    g.init(r, ux, uy)
    return g, (r, ux, uy), dict(tau=tau, dt=dt, ds=ds, N=4), 9


CASES = {
    "cs": (bench_cs, 3, lb.LB_FP32, False),
    "fd": (bench_fd, 2, lb.LB_FP32, False),
    # the timed configuration: autotuned launch shapes, graph-replayed runs
    "cs_tuned": (bench_cs, 10, lb.LB_FP32, True),
    "fd_tuned": (bench_fd, 5, lb.LB_FP32, True),
    # the 4096^2 vortex in FP32 and FP16-shifted storage, D2Q36 at 2048^2
    "cs4096_fp32": (lambda: tgv4096_cs(lb.LB_FP32), 10, lb.LB_FP32, True),
    "cs4096_fp16": (lambda: tgv4096_cs(lb.LB_FP16_SHIFTED), 6, lb.LB_FP16_SHIFTED, False),
    "fd36": (tgv2048_fd36, 5, lb.LB_FP32, True),
}


@pytest.mark.parametrize("which", list(CASES))
def test_sampled_nodes_full_size(which):
    build, nsteps, prec, tuned = CASES[which]
    print("case: full size sampled nodes", which, nsteps, flush=True)
    g, (r, ux, uy), prm, reach = build()
    if tuned:
        g.autotune(3)
    g.step(nsteps)
    f = g.get_state()
    Nn = g.Nx
    R = reach * nsteps + 2
    W = 2 * R + 1
    rng = np.random.default_rng(2048)
    pts = [(0, 0), (Nn - 1, Nn - 1), (0, Nn - 1), (Nn - 1, 0), (Nn // 2 - 1, Nn // 2)] + \
        [tuple(p) for p in rng.integers(0, Nn, (10, 2))]
    worst = 0.0
    for (x, y) in pts:
        xs = (np.arange(x - R, x + R + 1)) % Nn
        ys = (np.arange(y - R, y + R + 1)) % Nn
        o = oracle.OracleSim(ORACLE_MODEL[g.model], W, W, prm["tau"], prm["dt"], prm["ds"], prm["N"])
        o.init(r[np.ix_(ys, xs)], ux[np.ix_(ys, xs)], uy[np.ix_(ys, xs)])
        o.step(nsteps)
        fo = o.get_state()[:, R, R]
        fg = f[:, y, x]
        tol = tolerance(prec, nsteps, fo[:, None, None], g.w, 1.0)
        err = float(np.max(np.abs(fg - fo)))
        worst = max(worst, err)
        assert err <= tol, (x, y, err, tol)
    print("worst sampled |df| = %.3e" % worst, flush=True)


@pytest.mark.parametrize("which", ["cs", "fd"])
def test_full_size_conservation_and_series(which):
    print("case: full size conservation", which, flush=True)
    g, _, _, _ = bench_cs() if which == "cs" else bench_fd()
    ax, ay, bx, by = workloads.separable_pattern("tgv", N, N)
    g.set_probe(ax, ay, bx, by)
    d0 = g.reduce()
    g.series_reserve(16)
    g.step_sampled(50, 10)
    rows = g.series_read()
    assert [int(t) for t in rows[:, 0]] == [0, 10, 20, 30, 40]
    d1 = g.reduce()
    # mass and momentum: FP32 storage rounding only (relative 2^-24 per value
    # per step, random signs): far below 1e-6 of the mass after 50 steps
    assert abs(d1[0] - d0[0]) <= 1e-6 * d0[0]
    assert abs(d1[1]) <= 1e-6 * d0[0] * 0.01 and abs(d1[2]) <= 1e-6 * d0[0] * 0.01
    # the fused sample at t = 0 equals the stand-alone reduction of the
    # initial state (FP32 per-node terms vs FP64 per-node terms)
    np.testing.assert_allclose(rows[0, 1:], d0, rtol=1e-6, atol=1e-9 * d0[0])
    # amplitude decays monotonically
    assert np.all(np.diff(rows[:, 5]) < 0) and d1[4] < rows[-1, 5]


def test_full_size_deterministic():
    print("case: full size determinism", flush=True)
    a, _, _, _ = bench_cs()
    b, _, _, _ = bench_cs()
    a.step(7)
    b.step(3)
    b.step(4)
    assert np.array_equal(a.get_state()[:, ::97, ::89], b.get_state()[:, ::97, ::89])
    ra, rb = a.reduce(), b.reduce()
    assert np.array_equal(ra, rb)
