"""The serving form: many simulations in one batched launch, admitted by
memory footprint while others run.  Each result must be the same alone and
in the mix, and the same as a single-simulation run of the same request."""
import math
import time

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1904_02471_amd import lb, serve, workloads

pytestmark = pytest.mark.gpu

EVERY = 10


def small_mix():
    """Seven requests of uneven size and model (the first is the probe)."""
    t = [{"kind": "tgv", "side": 96, "model": "cs", "tau_std": 0.7, "steps": 57},
         {"kind": "shear", "side": 64, "model": "fd16", "tau_std": 0.9, "steps": 33},
         {"kind": "tgv", "side": 200, "model": "cs", "tau_std": 0.55, "steps": 121},
         {"kind": "shear", "side": 128, "model": "cs", "tau_std": 1.3, "steps": 20},
         {"kind": "tgv", "side": 130, "model": "fd16", "tau_std": 0.6, "steps": 45},
         {"kind": "tgv", "side": 64, "model": "fd16", "tau_std": 1.1, "steps": 70},
         {"kind": "shear", "side": 300, "model": "cs", "tau_std": 0.8, "steps": 64}]
    return t


def run_server(entries, budget=8 << 30, slots=64, chunk=16):
    srv = serve.Server(budget, slots, chunk)
    fields = serve.field_cache()
    ids = []
    for i, e in enumerate(entries):
        kw = serve.trace_request(e, fields)
        ids.append(srv.submit(sample_every=EVERY, tag=i, **kw))
    res = serve.wait_all(srv, len(entries), 120)
    srv.close()
    by_tag = {r["tag"]: r for r in res}
    for r in res:
        assert r["status"] == 0, r
    return [by_tag[i] for i in range(len(entries))]


def single_run(e):
    """The same request through the single-simulation path."""
    kw = serve.trace_request(e, serve.field_cache())
    g = lb.Sim(kw["model"], kw["Nx"], kw["Ny"], kw["tau"], kw["dt"], kw["ds"], kw["N"], precision=lb.LB_FP32)
    g.init(kw["rho"], kw["ux"], kw["uy"])
    g.set_probe(*kw["probe"])
    g.series_reserve(kw["nsteps"] // EVERY + 2)
    g.step_sampled(kw["nsteps"], EVERY)
    rows = g.series_read()
    final = np.concatenate([[kw["nsteps"]], g.reduce()])
    return np.vstack([rows, final])


def test_alone_equals_in_the_mix():
    """Served results equal alone and in a mix, and equal the single-simulation
    path bit for bit."""
    print("case: serving alone vs mix", flush=True)
    mix = small_mix()
    alone = run_server([mix[0]])[0]
    together = run_server(mix)
    assert np.array_equal(alone["samples"], together[0]["samples"])
    # and every member of the mix equals its single-simulation run
    for e, r in zip(mix, together):
        ref = single_run(e)
        assert r["samples"].shape == ref.shape, (e, r["samples"].shape, ref.shape)
        assert np.array_equal(r["samples"], ref), e
        assert r["t_finish"] >= r["t_admit"] >= r["t_submit"]


def test_served_result_matches_oracle():
    print("case: serving vs oracle", flush=True)
    e = {"kind": "tgv", "side": 40, "model": "fd16", "tau_std": 0.8, "steps": 30}
    c = {"kind": "shear", "side": 48, "model": "cs", "tau_std": 0.7, "steps": 40}
    res = run_server([e, c])
    for ent, r in zip([e, c], res):
        kw = serve.trace_request(ent, serve.field_cache())
        om = oracle.FD_D2Q16 if kw["model"] == lb.LB_FD_D2Q16 else oracle.CS_D2Q9
        o = oracle.OracleSim(om, kw["Nx"], kw["Ny"], kw["tau"], kw["dt"], kw["ds"], kw["N"])
        o.init(kw["rho"], kw["ux"], kw["uy"])
        ax, ay, bx, by = kw["probe"]
        px, py = np.outer(ay, ax), np.outer(by, bx)
        o.step(kw["nsteps"])
        want = o.reduce(px, py)
        got = r["samples"][-1]
        assert got[0] == kw["nsteps"]
        assert got[1] == pytest.approx(want[0], rel=1e-6)
        assert got[4] == pytest.approx(want[3], rel=1e-4)
        assert got[5] == pytest.approx(want[4], rel=1e-5)


def test_admission_by_memory_budget():
    print("case: serving budget", flush=True)
    entries = [{"kind": "tgv", "side": 256, "model": "cs", "tau_std": 0.7, "steps": 30 + 5 * i} for i in range(6)]
    one = 2 * 9 * 256 * 256 * 4
    res = run_server(entries, budget=int(1.5 * one) + (1 << 20), slots=64, chunk=8)
    # only one simulation fits at a time: admissions follow completions
    order = sorted(res, key=lambda r: r["t_admit"])
    for a, b in zip(order, order[1:]):
        assert b["t_admit"] >= a["t_finish"] - 1e-3
    srv = serve.Server(1 << 20, 4, 8)
    with pytest.raises(lb.LBError) as err:
        kw = serve.trace_request(entries[0], serve.field_cache())
        srv.submit(sample_every=EVERY, **kw)
    assert err.value.code == lb.LB_EBUSY
    with pytest.raises(lb.LBError) as err:
        kw = serve.trace_request(entries[0], serve.field_cache())
        kw["tau"] = 0.3   # negative viscosity
        srv.submit(sample_every=EVERY, **kw)
    assert err.value.code == lb.LB_EINVAL
    srv.close()


def run_server_cfg(entries, use_graphs, tune_tiles=True, chunk=16):
    srv = serve.Server(8 << 30, 64, chunk, use_graphs=use_graphs, tune_tiles=tune_tiles)
    fields = serve.field_cache()
    for i, e in enumerate(entries):
        srv.submit(sample_every=EVERY, tag=i, **serve.trace_request(e, fields))
    res = serve.wait_all(srv, len(entries), 120)
    srv.close()
    by_tag = {r["tag"]: r for r in res}
    return [by_tag[i] for i in range(len(entries))]


def test_graph_replay_equals_plain_launches():
    """The captured batched step replays exactly the kernels launched one by
    one: bitwise the same series, whatever later-stage tile height the
    tuner picked."""
    print("case: serving graphs vs plain launches", flush=True)
    mix = small_mix()
    g = run_server_cfg(mix, True)
    p = run_server_cfg(mix, False, tune_tiles=False)
    for e, a, b in zip(mix, g, p):
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["samples"], b["samples"]), e


def test_admission_while_running():
    """Requests submitted after the first batched chunk has started join the
    running batch (admitted before the earlier requests finish) and give the
    single-simulation results bit for bit."""
    print("case: serving mid-run admission", flush=True)
    first = [{"kind": "tgv", "side": 256, "model": "cs", "tau_std": 0.6, "steps": 400},
             {"kind": "tgv", "side": 128, "model": "fd16", "tau_std": 0.8, "steps": 120}]
    late = [{"kind": "shear", "side": 96, "model": "fd16", "tau_std": 0.7, "steps": 37},
            {"kind": "tgv", "side": 160, "model": "cs", "tau_std": 0.9, "steps": 51}]
    srv = serve.Server(8 << 30, 64, 8)
    fields = serve.field_cache()
    for i, e in enumerate(first):
        srv.submit(sample_every=EVERY, tag=i, **serve.trace_request(e, fields))
    t_end = time.time() + 60
    while srv.stats()["batch_steps"] < 1:
        assert time.time() < t_end, "no batched step launched"
        time.sleep(1e-3)
    for i, e in enumerate(late):
        srv.submit(sample_every=EVERY, tag=len(first) + i, **serve.trace_request(e, fields))
    res = {r["tag"]: r for r in serve.wait_all(srv, len(first) + len(late), 120)}
    srv.close()
    entries = first + late
    for i, e in enumerate(entries):
        assert res[i]["status"] == 0
        assert np.array_equal(res[i]["samples"], single_run(e)), e
    # the late requests ran beside the first ones
    assert min(res[i]["t_admit"] for i in (2, 3)) < res[0]["t_finish"]


def test_apparent_viscosity_of_results():
    """nu_app of a served result: the library's FP64 fit of its amplitude
    series against the oracle package's fit of the same series."""
    print("case: serving nu_app", flush=True)
    ents = [{"kind": "tgv", "side": 64, "model": "cs", "tau_std": 0.7, "steps": 300},
            {"kind": "shear", "side": 64, "model": "fd16", "tau_std": 0.8, "steps": 200}]
    srv = serve.Server(8 << 30, 64, 16)
    fields = serve.field_cache()
    ks = []
    for i, e in enumerate(ents):
        kw = serve.trace_request(e, fields)
        k = 2 * math.pi / e["side"] if e["model"] == "cs" else 2 * math.pi
        k2 = 2 * k * k if e["kind"] == "tgv" else k * k
        ks.append(k)
        srv.submit(sample_every=EVERY, tag=i, decay_k2=k2, **kw)
    res = {r["tag"]: r for r in serve.wait_all(srv, len(ents), 120)}
    srv.close()
    for i, e in enumerate(ents):
        kw = serve.trace_request(e, fields)
        s = res[i]["samples"]
        want = exact.apparent_viscosity(s[:, 0] * kw["dt"], s[:, 5], ks[i], e["kind"])
        nu = res[i]["nu_app"]
        print("%s %s nu_app %.9e oracle fit %.9e" % (e["model"], e["kind"], nu, want), flush=True)
        assert nu == pytest.approx(want, rel=1e-10)
        # and close to the viscosity the request was set up with
        nu0 = (e["tau_std"] - 0.5) / 3.0 if e["model"] == "cs" else kw["tau"]
        assert nu == pytest.approx(nu0, rel=0.05)


def unstable_cs_request(n=32, seed=5):
    """A CS request that blows up: tau = 0.5002 (omega near 2) and a random
    state at up to 0.45 of the lattice speed; the FP64 oracle's populations
    reach 1e12 after 25 steps and 1e28 after 50, so FP32 overflows within
    ~60 steps and the diagnostics turn non-finite."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (n, n))
    ux, uy = rng.uniform(-0.45, 0.45, (2, n, n))
    return dict(model=lb.LB_CS_D2Q9, Nx=n, Ny=n, tau=0.5002, dt=1.0, ds=1.0, N=2, rho=rho, ux=ux, uy=uy,
                nsteps=200)


def test_a_diverging_request_fails_alone():
    """A request whose state overflows is reported with LB_ENAN and no
    samples; the requests beside it in the batch, and one submitted after it,
    give their single-simulation results bit for bit.  (Non-finite values are
    ordinary arithmetic here: no kernel indexes by a state value.)"""
    print("case: serving diverging request", flush=True)
    good = [{"kind": "tgv", "side": 64, "model": "cs", "tau_std": 0.7, "steps": 120},
            {"kind": "shear", "side": 64, "model": "fd16", "tau_std": 0.8, "steps": 60}]
    fields = serve.field_cache()
    srv = serve.Server(8 << 30, 64, 16)
    srv.submit(sample_every=EVERY, tag=0, **serve.trace_request(good[0], fields))
    srv.submit(sample_every=EVERY, tag=9, **unstable_cs_request())
    srv.submit(sample_every=EVERY, tag=1, **serve.trace_request(good[1], fields))
    res = {r["tag"]: r for r in serve.wait_all(srv, 3, 120)}
    later = {"kind": "tgv", "side": 96, "model": "cs", "tau_std": 0.9, "steps": 40}
    srv.submit(sample_every=EVERY, tag=2, **serve.trace_request(later, fields))
    res.update({r["tag"]: r for r in serve.wait_all(srv, 1, 120)})
    srv.close()
    assert res[9]["status"] == lb.LB_ENAN and res[9]["samples"].shape[0] == 0
    assert math.isnan(res[9]["nu_app"])
    for tag, e in ((0, good[0]), (1, good[1]), (2, later)):
        assert res[tag]["status"] == 0
        assert np.array_equal(res[tag]["samples"], single_run(e)), e
    # the single-simulation path reports the same condition
    kw = unstable_cs_request()
    g = lb.Sim(kw["model"], kw["Nx"], kw["Ny"], kw["tau"], kw["dt"], kw["ds"], kw["N"])
    g.init(kw["rho"], kw["ux"], kw["uy"])
    g.step(kw["nsteps"])
    with pytest.raises(lb.LBError) as err:
        g.reduce()
    assert err.value.code == lb.LB_ENAN


def test_node_limit_admits_in_arrival_order():
    """With a limit on the nodes in flight the server admits queued requests
    in arrival order only while the admitted grids fit the limit (a request
    larger than it alone), and every result still equals its single run bit
    for bit; the limit is set before the first submission only."""
    print("case: serving node limit", flush=True)
    entries = [{"kind": "tgv", "side": 64, "model": "cs", "tau_std": 0.7, "steps": 90},
               {"kind": "shear", "side": 64, "model": "fd16", "tau_std": 0.9, "steps": 30},
               {"kind": "tgv", "side": 64, "model": "fd16", "tau_std": 0.6, "steps": 20},
               {"kind": "tgv", "side": 96, "model": "cs", "tau_std": 0.8, "steps": 40},
               {"kind": "shear", "side": 64, "model": "cs", "tau_std": 1.2, "steps": 25}]
    srv = serve.Server(8 << 30, 64, 8, node_limit=2 * 64 * 64)
    fields = serve.field_cache()
    for i, e in enumerate(entries):
        srv.submit(sample_every=EVERY, tag=i, **serve.trace_request(e, fields))
    assert serve._lib.lb_server_set_node_limit(srv._h, 0) == lb.LB_ESTATE
    peak = 0
    t_end = time.time() + 120
    res = {}
    while len(res) < len(entries):
        assert time.time() < t_end, "results missing"
        peak = max(peak, srv.stats()["running"])
        for r in srv.poll(16, 1000):
            res[r["tag"]] = r
    srv.close()
    assert peak <= 2
    for i, e in enumerate(entries):
        assert res[i]["status"] == 0
        assert np.array_equal(res[i]["samples"], single_run(e)), e
    # arrival order: the third request waits for one of the first two, the
    # 96^2 request (above the limit with anything else) runs alone
    assert res[2]["t_admit"] >= min(res[0]["t_finish"], res[1]["t_finish"])
    others = [res[i] for i in (0, 1, 2, 4)]
    assert all(o["t_finish"] <= res[3]["t_admit"] or o["t_admit"] >= res[3]["t_finish"] for o in others)


def test_shortest_first_admission():
    """LB_ADMIT_SHORTEST admits the queued request of smallest estimated work
    (nodes x steps x the model's cost) first: with one simulation at a time,
    the requests queued behind the first one finish in order of their work,
    and every result equals its single run bit for bit."""
    print("case: serving shortest first", flush=True)
    entries = [{"kind": "tgv", "side": 64, "model": "cs", "tau_std": 0.7, "steps": 60},      # work 64^2 x 60
               {"kind": "tgv", "side": 64, "model": "fd16", "tau_std": 0.9, "steps": 40},    # x 12 x 40
               {"kind": "shear", "side": 64, "model": "cs", "tau_std": 1.1, "steps": 20},    # 20
               {"kind": "tgv", "side": 64, "model": "cs", "tau_std": 0.8, "steps": 200},     # 200
               {"kind": "shear", "side": 64, "model": "fd16", "tau_std": 0.6, "steps": 5}]   # 60
    srv = serve.Server(8 << 30, 64, 8, node_limit=64 * 64, policy=serve.ADMIT_SHORTEST)
    assert serve._lib.lb_server_set_policy(srv._h, 0) == lb.LB_OK  # before the first submission
    assert serve._lib.lb_server_set_policy(srv._h, 2) == lb.LB_EINVAL
    assert serve._lib.lb_server_set_policy(srv._h, serve.ADMIT_SHORTEST) == lb.LB_OK
    fields = serve.field_cache()
    kws = [serve.trace_request(e, fields) for e in entries]  # prepared first: the submissions follow at once
    for i, kw in enumerate(kws):
        srv.submit(sample_every=EVERY, tag=i, **kw)
    assert serve._lib.lb_server_set_policy(srv._h, 0) == lb.LB_ESTATE
    res = {r["tag"]: r for r in serve.wait_all(srv, len(entries), 120)}
    srv.close()
    for i, e in enumerate(entries):
        assert res[i]["status"] == 0
        assert np.array_equal(res[i]["samples"], single_run(e)), e
    work = {i: 64 * 64 * e["steps"] * (12.0 if e["model"] == "fd16" else 1.0) for i, e in enumerate(entries)}
    # the first request may be admitted before the others arrive; the rest
    # run one at a time in order of work (ties: arrival)
    later = sorted((i for i in range(len(entries)) if res[i]["t_admit"] > min(r["t_admit"] for r in res.values())),
                   key=lambda i: res[i]["t_admit"])
    assert [work[i] for i in later] == sorted(work[i] for i in later), later
