"""GPU runs at the largest grids lb_create accepts, where the 32-bit
byte offsets of the FD buffer resources and the 32-bit node counters come
closest to their limits: CS D2Q9 with Nx * Ny = 2^30 nodes, and FD D2Q9 with
population and moment planes 126,720 bytes short of 4 GiB (32768 x 32767
FP32).  The state varies from node to node in both directions
(workloads.separable_random_state), so a read from a wrong row or column
shows; sampled nodes, the grid's corners and last rows among them, are
checked against the oracle on a periodic window around each (moments: the
full state would need 77 GB of host memory).  Device memory: 77 GB (CS),
155 GB (FD) plus the transfer buffers."""
import time

import numpy as np
import pytest

import oracle
from paper_1904_02471_amd import lb, units, workloads
from tests.gpu_helpers import ORACLE_MODEL, tolerance

pytestmark = pytest.mark.gpu


def log(t0, msg):
    print("  %6.1f s  %s" % (time.time() - t0, msg), flush=True)


def make(model, Nx, Ny, tau, dt, ds, N):
    try:
        return lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=lb.LB_FP32)
    except lb.LBError as e:
        if e.code == lb.LB_ENOMEM:
            pytest.skip("not enough device memory for the %d x %d grid" % (Nx, Ny))
        raise


def check_samples(g, window, prm, nsteps, reach, t0):
    """Moments of sampled nodes against the oracle on a periodic window
    wider than the steps' reach."""
    Nx, Ny, K = g.Nx, g.Ny, g.K
    rho, ux, uy = g.moments()
    log(t0, "moments read")
    R = reach * nsteps + 2
    W = 2 * R + 1
    rng = np.random.default_rng(30)
    pts = [(0, 0), (Nx - 1, Ny - 1), (0, Ny - 1), (Nx - 1, 0), (Nx // 2, Ny - 2), (Nx - 33, Ny - 17)] + \
        [tuple(int(v) for v in p) for p in zip(rng.integers(0, Nx, 8), rng.integers(0, Ny, 8))]
    vmax = float(max(np.max(np.abs(g.vx)), np.max(np.abs(g.vy))))
    worst = 0.0
    for (x, y) in pts:
        xs = np.arange(x - R, x + R + 1) % Nx
        ys = np.arange(y - R, y + R + 1) % Ny
        o = oracle.OracleSim(ORACLE_MODEL[g.model], W, W, prm["tau"], prm["dt"], prm["ds"], prm["N"])
        o.init(*window(ys, xs))
        o.step(nsteps)
        fo = o.get_state()[:, R, R]
        ro, xo, yo = (m[R, R] for m in o.moments())
        tf = tolerance(lb.LB_FP32, nsteps, fo[:, None, None], g.w, 1.0)
        tr = K * tf
        tu = (K * vmax * tf + abs(max(abs(xo), abs(yo))) * tr) / (ro - tr)
        er, eu = abs(rho[y, x] - ro), max(abs(ux[y, x] - xo), abs(uy[y, x] - yo))
        worst = max(worst, er / tr, eu / tu)
        assert er <= tr and eu <= tu, ((x, y), er, tr, eu, tu)
    log(t0, "%d sampled nodes within the bound (worst %.2f of it)" % (len(pts), worst))


def test_cs_at_two_to_the_thirty_nodes():
    print("case: max size cs 32768 x 32768 fp32", flush=True)
    t0 = time.time()
    n = 32768
    g = make(lb.LB_CS_D2Q9, n, n, 0.7, 1.0, 1.0, 2)
    rho, ux, uy, window = workloads.separable_random_state(n, n, 2030)
    log(t0, "fields ready")
    g.init(rho, ux, uy)
    del rho, ux, uy
    log(t0, "initialised")
    g.step(2)
    g.synchronize()
    log(t0, "2 steps")
    check_samples(g, window, dict(tau=0.7, dt=1.0, ds=1.0, N=2), 2, 1, t0)
    g.destroy()


def test_fd_planes_just_under_four_gib():
    print("case: max size fd d2q9 32768 x 32767 fp32", flush=True)
    t0 = time.time()
    Nx, Ny = 32768, 32767
    ds = 1.0 / Nx
    tau = 1e-5
    dt = units.fd_time_step(tau, ds, lb.lb_model_info(lb.LB_FD_D2Q9)[0].max(), 0.5)
    g = make(lb.LB_FD_D2Q9, Nx, Ny, tau, dt, ds, 2)
    rho, ux, uy, window = workloads.separable_random_state(Nx, Ny, 2031)
    log(t0, "fields ready")
    g.init(rho, ux, uy)
    del rho, ux, uy
    log(t0, "initialised")
    g.step(1)
    g.synchronize()
    log(t0, "1 step (3 stage launches)")
    check_samples(g, window, dict(tau=tau, dt=dt, ds=ds, N=2), 1, 9, t0)
    g.destroy()
