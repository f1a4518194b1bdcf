"""Benchmark of the lattice Boltzmann hot path on one MI355X.

One step = one collision-streaming D2Q9 step and one finite-difference
D2Q16 step (three Runge-Kutta stage launches) on a Taylor-Green vortex,
each with the FP64 diagnostics fused into the step kernels every 10th step;
the timed region runs the K steps of the CS simulation, then the K steps of
the FD one (independent simulations).
Default workload: 2048 x 2048 periodic, rho0 = 1, u0 = 0.01 (standard
lattice units), CS tau = 0.6, FD D2Q16 with N = 3 at the same viscosity
(tau_FD = (tau - 1/2) / (sqrt(3) N)), dt_FD = min(CFL 0.5, tau_FD), FP32
storage.  Inputs are resident in HBM before the timed region.

Prints one JSON line: MLUPS of the whole step (node updates per second:
one update advances a node by one CS step and one FD step), per-model MLUPS
and HBM fractions, the roofline of the dominant kernel (the FD stage), the
CS step at 4096^2 with FP32 and FP16-shifted storage (states larger than the
last-level cache, so those byte rates are HBM rates), the FD D2Q36 step at
2048^2, the serving stream,
and the FP64 CPU oracle timed on bounded samples of the same workload (all
usable host threads, and one thread).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Published FP32 vector peak of MI355X: 256 CUs x 4 SIMDs x 2.4 GHz x 64 fmas
# per SIMD and quad-cycle.  Plain (non-packed) FP32 instructions can reach
# it: a SIMD co-issues the VALU instructions of two waves in one quad-cycle
# when neither reads an SGPR and their VGPR operands allow it (FMA chains
# over VGPR operands measured 110-131 TFLOP/s with this build's flags).
VALU_PEAK_PUBLISHED_TFLOPS = 157.3
# Algorithmic flops of the FD D2Q16 (N = 3) stage, fma counted as 2: per
# node and population the x- and y-face WENO-5 values (47 each, with the
# second differences, smoothness terms and first differences of a cell
# shared by its two faces), the two flux differences (2), the order-3
# equilibrium (29) and the stage update (8 in stage 1, 11 with the
# Runge-Kutta combination of stages 2 and 3); per node the moments of 16
# populations (80) and the moment-exact equilibrium corrections (40).
FD16_FLOPS_NODE_POP = (2 * 47 + 2 + 29 + 8, 2 * 47 + 2 + 29 + 11, 2 * 47 + 2 + 29 + 11)
FD16_FLOPS_NODE = 120


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--sample-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cache-free", action="store_true",
                    help="skip the 4096^2 CS FP32 / FP16 runs (state larger than the last-level cache) "
                         "and the 2048^2 FD D2Q36 run")
    ap.add_argument("--only", choices=["cs", "fd"], default=None,
                    help="time one model alone (profiling runs); the JSON line is then per model")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a plain device copy of the CS state size (counter calibration)")
    ap.add_argument("--fd-fused", type=int, default=-1,
                    help="FD step form after autotuning: -1 the tuner's choice, 0 the three stage launches, "
                         "R > 0 the temporally blocked step with R-row segments (profiling runs)")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the serving stream to replay (0: skip; 512: the whole stream)")
    ap.add_argument("--serving-node-limit", type=int, default=1 << 24,
                    help="grid nodes of the simulations the server admits at once (0: no limit; default "
                         "2^24, a 4096^2 grid's worth, which fills the device)")
    ap.add_argument("--serving-policy", choices=["arrival", "shortest"], default="arrival",
                    help="admission order of the server (arrival order, or smallest estimated work first)")
    ap.add_argument("--serving-batched-only", action="store_true",
                    help="replay the stream batched only, without the one-simulation-per-launch comparison "
                         "(profiling runs)")
    return ap.parse_args()


def make_sims(lb, workloads, units, n, stream):
    u0 = 0.01
    cs = lb.Sim(lb.LB_CS_D2Q9, n, n, 0.6, 1.0, 1.0, 2, precision=lb.LB_FP32)
    r, ux, uy, _ = workloads.taylor_green(n, n, u0, 1.0 / 3.0)
    cs.set_stream(stream)
    cs.init(r, ux, uy)
    ax, ay, bx, by = workloads.separable_pattern("tgv", n, n)
    cs.set_probe(ax, ay, bx, by)

    ds = 1.0 / n
    tau_fd = units.tau_fd_from_std(0.6, n)
    vmax = lb.lb_model_info(lb.LB_FD_D2Q16)[0].max()
    dt_fd = units.fd_time_step(tau_fd, ds, vmax, 0.5)
    fd = lb.Sim(lb.LB_FD_D2Q16, n, n, tau_fd, dt_fd, ds, 3, precision=lb.LB_FP32)
    r, ux, uy, _ = workloads.taylor_green(n, n, units.velocity_fd_from_std(u0), 1.0)
    fd.set_stream(stream)
    fd.init(r, ux, uy)
    fd.set_probe(ax, ay, bx, by)
    return cs, fd, {"tau_fd": tau_fd, "dt_fd": dt_fd}


def cache_free_cs(lb, workloads, stream, n=4096, steps=200, warmup=20):
    """CS D2Q9 plain steps on the n x n Taylor-Green vortex (tau = 0.55) with
    FP32, FP16-shifted and FP16 reference-shifted storage: at 4096^2 the two
    state buffers (1.2 GB / 0.6 GB) exceed the 256 MB last-level cache, so the
    byte rate is the HBM rate.  Bytes per node-step: 2 x 9 stored values, plus
    the 4-byte reference velocity of the reference-shifted form.  Autotuned
    launch shapes; plain steps as the library runs them."""
    import torch
    out = {"grid": [n, n], "steps": steps}
    for name, prec, s in (("fp32", lb.LB_FP32, 4), ("fp16_shifted", lb.LB_FP16_SHIFTED, 2),
                          ("fp16_ref", lb.LB_FP16_REF, 2)):
        sim = lb.Sim(lb.LB_CS_D2Q9, n, n, 0.55, 1.0, 1.0, 2, precision=prec)
        sim.set_stream(stream.cuda_stream)
        r, ux, uy, _ = workloads.taylor_green(n, n, 0.01, 1.0 / 3.0)
        sim.init(r, ux, uy)
        del r, ux, uy
        threads = sim.autotune(10)[0]
        nt = sim.cs_nontemporal()
        sim.step(warmup)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            sim.step(steps)
            b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        bpn = 18 * s + (4 if prec == lb.LB_FP16_REF else 0)
        gbs = bpn * n * n / (ms * 1e-3) / 1e9
        out[name] = {"ms_per_step": round(ms, 5), "mlups": round(n * n / (ms * 1e-3) / 1e6, 1),
                     "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_node_step": bpn, "cs_threads": threads, "cs_nontemporal_stores": nt}
        sim.destroy()
    return out


def host_boundary(lb, workloads, units, sims, n, K):
    """Cost of the C ABI's host buffers around a K-step job on the n x n
    workload: lb_init from host rho, u (3 FP64 fields, 24 B per node up,
    plus the equilibrium initialisation) and lb_moments back to host (24 B
    per node down, plus the moments kernel), wall clock with the device
    idle before each call, second of two calls.  `pcie_inclusive_mlups` is
    the job's rate with both transfers counted: nodes x K / (t_init + K x
    t_step + t_moments); it is never the headline value (whose inputs are
    resident in HBM).  Re-initialises the simulations (after the timed
    steps)."""
    import torch
    out = {}
    nodes = n * n
    fields = {"cs_d2q9": workloads.taylor_green(n, n, 0.01, 1.0 / 3.0)[:3],
              "fd_d2q16": workloads.taylor_green(n, n, units.velocity_fd_from_std(0.01), 1.0)[:3]}
    for name, sim, step_ms in sims:
        r, ux, uy = fields[name]
        t_init = t_mom = 0.0
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.init(r, ux, uy)
            sim.synchronize()
            t1 = time.perf_counter()
            sim.moments()
            t2 = time.perf_counter()
            t_init, t_mom = (t1 - t0) * 1e3, (t2 - t1) * 1e3
        job_ms = t_init + K * step_ms + t_mom
        out[name] = {"init_ms": round(t_init, 3), "moments_ms": round(t_mom, 3),
                     "bytes_up": 24 * nodes, "bytes_down": 24 * nodes,
                     "steps": K, "pcie_inclusive_mlups": round(nodes * K / (job_ms * 1e-3) / 1e6, 1),
                     "resident_mlups": round(nodes / (step_ms * 1e-3) / 1e6, 1)}
    return out


def fd_d2q36(lb, workloads, units, stream, n=2048, steps=60, warmup=8):
    """FD D2Q36 (N = 4) plain steps on the n x n Taylor-Green vortex of the
    D2Q36 workload (tau_FD = 5e-4, dt at CFL 0.5), FP32 storage, autotuned.
    The warm-up replays the 4-step graph twice, so that its capture (after
    the tuner's shape change) stays out of the timed steps."""
    import torch
    ds = 1.0 / n
    tau = 5e-4
    vmax = lb.lb_model_info(lb.LB_FD_D2Q36)[0].max()
    dt = units.fd_time_step(tau, ds, vmax, 0.5)
    sim = lb.Sim(lb.LB_FD_D2Q36, n, n, tau, dt, ds, 4, precision=lb.LB_FP32)
    sim.set_stream(stream.cuda_stream)
    r, ux, uy, _ = workloads.taylor_green(n, n, 0.01, 1.0)
    sim.init(r, ux, uy)
    del r, ux, uy
    shapes = sim.autotune(3)
    sim.step(warmup)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        a.record(stream)
        sim.step(steps)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    sim.destroy()
    gbs = 8 * 36 * 4 * n * n / (ms * 1e-3) / 1e9
    return {"grid": [n, n], "steps": steps, "tau_fd": tau, "dt_fd": dt, "ms_per_step": round(ms, 5),
            "mlups": round(n * n / (ms * 1e-3) / 1e6, 1), "achieved_gbs_stagewise": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node_step": 8 * 36 * 4,
            "fd_tile_rows": shapes[1], "fd_tile_rows_later_stages": shapes[2]}


def fd_fused_compare(lb, workloads, units, stream, n=2048, steps=40, warmup=8):
    """FD D2Q16 (N = 3) plain steps on the n x n vortex of the benchmark: the
    three stage launches (autotuned tiles) against the temporally blocked
    step with 32-, 64- and 128-row segments; MLUPS and the HBM rate of each
    form's algorithmic bytes (stage launches 8 K s per step, fused 2 K s plus
    the moment planes).  D2Q36 has no fused form (its register windows do not
    fit), so only D2Q9/D2Q16 are timed.  Each form's warm-up replays its
    graph at least once, keeping the capture out of the timed steps."""
    import torch
    ds = 1.0 / n
    tau = units.tau_fd_from_std(0.6, n)
    vmax = lb.lb_model_info(lb.LB_FD_D2Q16)[0].max()
    dt = units.fd_time_step(tau, ds, vmax, 0.5)
    sim = lb.Sim(lb.LB_FD_D2Q16, n, n, tau, dt, ds, 3, precision=lb.LB_FP32)
    sim.set_stream(stream.cuda_stream)
    r, ux, uy, _ = workloads.taylor_green(n, n, units.velocity_fd_from_std(0.01), 1.0)
    sim.init(r, ux, uy)
    del r, ux, uy
    sim.autotune(3)
    out = {"grid": [n, n], "steps": steps}
    for name, ys in (("stage_launches", 0), ("fused_ys32", 32), ("fused_ys64", 64), ("fused_ys128", 128)):
        sim.set_fd_fused(ys)
        sim.step(warmup)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            sim.step(steps)
            b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        bpn = 512 if ys == 0 else 2 * 16 * 4 + 24
        gbs = bpn * n * n / (ms * 1e-3) / 1e9
        out[name] = {"ms_per_step": round(ms, 5), "mlups": round(n * n / (ms * 1e-3) / 1e6, 1),
                     "bytes_per_node_step": bpn, "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    sim.destroy()
    out["fd_d2q36"] = "stage launches only: 36 populations of register windows exceed the register file"
    return out


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1904_02471_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_record(kernel, n, shape=None):
    """The counter record of `kernel` on the n x n workload in
    paper_1904_02471_amd/kernel_traffic.json (calibrated FETCH_SIZE +
    WRITE_SIZE bytes and SQ_INSTS_VALU per launch), or None when none was
    recorded for this workload and launch shape, or the kernel's sources
    changed since."""
    path = os.path.join(ROOT, "paper_1904_02471_amd", "kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec or rec.get("grid") != [n, n] or rec.get("sources_sha256") != source_digest(rec["sources"]):
        return None
    for key, want in (shape or {}).items():
        if rec.get(key) != want:
            return None
    return rec


def fd_stage_record(n, rows_first, rows_later):
    """Counter figures of an FD stage launch on the n x n workload for the
    tuned tile heights: the recorded first-stage instance with rows_first
    rows per thread and the later-stage one with rows_later, averaged over
    the three launches of a step (one first, two later).  None when either
    instance has no record, or the kernel's sources changed since."""
    rec = kernel_record("fd_stage_kernel", n)
    if not rec:
        return None
    inst = rec.get("instances", {})
    a, b = inst.get("stage1_rows%d" % rows_first), inst.get("stage23_rows%d" % rows_later)
    if not a or not b:
        return None
    out = {"bytes_per_launch": (a["bytes"] + 2 * b["bytes"]) / 3.0}
    for key in ("valu_insts", "valu_pairs"):
        if key in a and key in b:
            out[key + "_per_launch"] = (a[key] + 2 * b[key]) / 3.0
    return out


def valu_issue(rec, launch_ms):
    """Vector-ALU issue of a launch, from its recorded counters over the
    quad-cycles of 1024 SIMDs at the nominal 2.4 GHz for the launch time
    measured here: instructions per SIMD and quad-cycle (at most 2, two
    waves co-issuing), the share of quad-cycles that issued at least one
    (SQ_INSTS_VALU less SQ_ACTIVE_INST_VALU2, the quad-cycles that issued
    two) and the share of instructions issued in pairs."""
    if not rec or "valu_insts_per_launch" not in rec:
        return None
    quads = 1024 * 2.4e9 / 4 * launch_ms * 1e-3
    insts = rec["valu_insts_per_launch"]
    out = {"insts_per_quad_cycle": round(insts / quads, 4)}
    pairs = rec.get("valu_pairs_per_launch")
    if pairs is not None:
        out["busy_frac"] = round((insts - pairs) / quads, 4)
        out["paired_share"] = round(2 * pairs / insts, 4)
    return out


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and the threads this
    process may use, capped at the 16 host threads a one-GPU machine shares."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail, max(1, min(16, avail))


def cpu_baseline(every, n):
    """FP64 oracle timed on the host on bounded samples of the same workload:
    the row-parallel mode on all usable host threads (bitwise the serial
    run) on the n x n grid itself, 2 CS D2Q9 steps + 1 FD D2Q16 step; and
    the plain serial run on 1024^2 x 3 CS steps + 512^2 x 2 FD steps (same
    work per node).  Diagnostics every `every` steps as on the GPU.  value =
    node updates per second of the all-thread run, one update = one CS step
    plus one FD step per node: 1 / (t_cs + t_fd) per node."""
    import oracle
    from paper_1904_02471_amd import units, workloads

    def run(model, m, steps, threads):
        if model == oracle.CS_D2Q9:
            s = oracle.OracleSim(model, m, m, 0.6, 1.0, 1.0, 2)
            r, ux, uy, (px, py) = workloads.taylor_green(m, m, 0.01, 1.0 / 3.0)
        else:
            ds = 1.0 / m
            tau = units.tau_fd_from_std(0.6, m)
            s = oracle.OracleSim(model, m, m, tau, units.fd_time_step(tau, ds, 2.3344142183389773, 0.5), ds, 3)
            r, ux, uy, (px, py) = workloads.taylor_green(m, m, units.velocity_fd_from_std(0.01), 1.0)
        s.set_threads(threads)
        s.init(r, ux, uy)
        del r, ux, uy
        t0 = time.perf_counter()
        for i in range(steps):
            if i % every == 0:
                s.reduce(px, py)
            s.step(1)
        t = (time.perf_counter() - t0) / (m * m * steps)
        s.close()
        return t

    model_name, avail, threads = host_cpu()
    t_cs = run(oracle.CS_D2Q9, n, 2, threads)
    t_fd = run(oracle.FD_D2Q16, n, 1, threads)
    s_cs = run(oracle.CS_D2Q9, 1024, 3, 1)
    s_fd = run(oracle.FD_D2Q16, 512, 2, 1)
    return {"value": 1e-6 / (t_cs + t_fd), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "FP64 C oracle, row-parallel on %d host threads (bitwise the serial run): CS D2Q9 TGV "
                      "%dx%d x 2 steps (%.3f MLUPS) + FD D2Q16 TGV %dx%d x 1 step (%.4f MLUPS); value = "
                      "1 / (t_cs + t_fd) per node" % (threads, n, n, 1e-6 / t_cs, n, n, 1e-6 / t_fd),
            "cpu_model": model_name, "host_threads_available": avail,
            "single_thread": {"value": 1e-6 / (s_cs + s_fd), "unit": "MLUPS", "cores": 1,
                              "sample": "serial: CS D2Q9 TGV 1024x1024 x 3 steps (%.3f MLUPS) + FD D2Q16 TGV "
                                        "512x512 x 2 steps (%.4f MLUPS)" % (1e-6 / s_cs, 1e-6 / s_fd)}}


def decay_fit_args(entry, kw):
    """(decay_k2, omega) of a serving request's viscosity fit: the amplitude
    of a shear wave decays at nu k^2, of a Taylor-Green vortex at 2 nu k^2
    (k = 2 pi / side per lattice spacing for CS, 2 pi on the FD unit box);
    a vortex started from f = f_eq rings at omega = 2 k c_s, fitted along when
    the run spans at least two periods."""
    from paper_1904_02471_amd import lb
    cs_model = kw["model"] == lb.LB_CS_D2Q9
    k = 2 * math.pi / entry["side"] if cs_model else 2 * math.pi
    if entry["kind"] == "shear":
        return k * k, 0.0
    omega = 2 * k * (1 / math.sqrt(3) if cs_model else 1.0)
    return 2 * k * k, (omega if omega * kw["nsteps"] * kw["dt"] >= 4 * math.pi else 0.0)


def serving_bench(n_requests, every, batched_only=False, node_limit=0, policy=0):
    """Replay the first n_requests of the seeded serving stream (Poisson
    arrivals, mean gap 2 ms; square grids 64..1024; CS D2Q9 or FD D2Q16;
    500-5000 steps) twice on the GPU: batched (lb_server, continuous
    batching: batched launches replayed as captured graphs, admission on a
    second stream) and one simulation per launch sequence (lb_sim per
    request, in arrival order, each alone on the GPU).  Reports sims/s,
    p50/p99 time-to-result (completion minus arrival) and service time
    (completion minus admission), and each request's apparent viscosity (the
    library's FP64 fit of its amplitude series) alone and in the mix."""
    import numpy as np

    from paper_1904_02471_amd import lb, serve, workloads

    trace = workloads.serving_trace(n_requests, 1904)
    fields = serve.field_cache()
    reqs = [serve.trace_request(e, fields) for e in trace]
    fits = [decay_fit_args(e, kw) for e, kw in zip(trace, reqs)]
    n = len(trace)

    # batched, continuous admission
    srv = serve.Server(hbm_budget_bytes=200 << 30, max_slots=512, chunk_steps=32, node_limit=node_limit,
                       policy=policy)
    results = {}
    t0 = time.perf_counter()
    c0 = srv.clock()
    k = 0
    while len(results) < n:
        now = time.perf_counter() - t0
        while k < n and trace[k]["arrival_s"] <= now:
            srv.submit(sample_every=every, tag=k, decay_k2=fits[k][0], decay_omega=fits[k][1], **reqs[k])
            k += 1
        for r in srv.poll(256, 500):
            results[r["tag"]] = r
            if len(results) % 64 == 0:
                print("serving batched: %d/%d done at %.1f s" % (len(results), n, time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
    wall_b = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    lat_b = np.array([results[i]["t_finish"] - (c0 + trace[i]["arrival_s"]) for i in range(n)])
    svc_b = np.array([results[i]["t_finish"] - results[i]["t_admit"] for i in range(n)])
    assert all(results[i]["status"] == 0 for i in range(n))
    batched = {"sims_per_s": round(n / wall_b, 3), "wall_s": round(wall_b, 3),
               "p50_s": round(float(np.percentile(lat_b, 50)), 4), "p99_s": round(float(np.percentile(lat_b, 99)), 4),
               "service_p50_s": round(float(np.percentile(svc_b, 50)), 4),
               "service_p99_s": round(float(np.percentile(svc_b, 99)), 4),
               "mlups": round(sum(kw["Nx"] * kw["Ny"] * kw["nsteps"] for kw in reqs) / wall_b / 1e6, 1),
               "batch_steps": stats["batch_steps"]}
    batched["node_limit"] = node_limit
    batched["admission"] = "shortest estimated work first" if policy else "arrival order"
    if batched_only:
        return {"requests": n, "batched": batched}
    # the same stream batched with shortest-estimated-work-first admission
    # (the one-simulation-per-launch side below keeps arrival order, as the
    # batched line above)
    shortest = serving_bench(n_requests, every, True, node_limit, 1)["batched"] if policy == 0 else None

    # one simulation per launch sequence
    lat_s = np.zeros(n)
    svc_s = np.zeros(n)
    nu_alone = np.zeros(n)
    same = True
    t0 = time.perf_counter()
    for i, e in enumerate(trace):
        while time.perf_counter() - t0 < e["arrival_s"]:
            time.sleep(2e-4)
        ts = time.perf_counter()
        kw = reqs[i]
        g = lb.Sim(kw["model"], kw["Nx"], kw["Ny"], kw["tau"], kw["dt"], kw["ds"], kw["N"], precision=lb.LB_FP32)
        g.init(kw["rho"], kw["ux"], kw["uy"])
        g.set_probe(*kw["probe"])
        g.series_reserve(kw["nsteps"] // every + 2)
        g.step_sampled(kw["nsteps"], every)
        rows = g.series_read()
        fin = np.concatenate([[kw["nsteps"]], g.reduce()])
        g.destroy()
        lat_s[i] = time.perf_counter() - t0 - e["arrival_s"]
        svc_s[i] = time.perf_counter() - ts
        series = np.vstack([rows, fin])
        same = same and np.array_equal(series, results[i]["samples"])
        nu_alone[i] = serve.fit_decay(series[:, 0] * kw["dt"], series[:, 5], fits[i][1]) / fits[i][0]
        if (i + 1) % 64 == 0:
            print("serving one-by-one: %d/%d done at %.1f s" % (i + 1, n, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    wall_s = time.perf_counter() - t0
    nodes_steps = sum(kw["Nx"] * kw["Ny"] * kw["nsteps"] for kw in reqs)
    nu_mix = np.array([results[i]["nu_app"] for i in range(n)])
    # viscosity each request was set up with: CS nu = (tau - 1/2)/3 in
    # lattice units, FD nu = tau_FD on the unit box
    nu0 = np.array([(kw["tau"] - 0.5) / 3.0 if kw["model"] == lb.LB_CS_D2Q9 else kw["tau"] for kw in reqs])
    err = np.abs(nu_mix / nu0 - 1)

    def pct(a, q):
        return round(float(np.percentile(a, q)), 4)
    return {
        "requests": n, "stream": "seed 1904, Poisson arrivals mean 2 ms, side U{64..1024}, CS D2Q9 / FD D2Q16 "
                                  "50/50, tau U[0.55,1.5], steps U{500..5000}, FP32, diagnostics every %d" % every,
        "batched": batched,
        "batched_shortest_first": shortest,
        "one_sim_per_launch": {"sims_per_s": round(n / wall_s, 3), "wall_s": round(wall_s, 3),
                               "p50_s": pct(lat_s, 50), "p99_s": pct(lat_s, 99),
                               "service_p50_s": pct(svc_s, 50), "service_p99_s": pct(svc_s, 99),
                               "mlups": round(nodes_steps / wall_s / 1e6, 1)},
        "speedup_sims_per_s": round(wall_s / wall_b, 3),
        "results_identical": bool(same),
        "nu_app": {"fit": "FP64 least squares of ln A(t) (lb_fit_decay) over every sample; Taylor-Green runs "
                          "spanning two acoustic periods fit the ringing at 2 k c_s along",
                   "max_rel_diff_alone_vs_mix": float(np.max(np.abs(nu_mix / nu_alone - 1))),
                   "rel_err_vs_setup_nu_p50": float(np.percentile(err, 50)),
                   "rel_err_vs_setup_nu_p99": float(np.percentile(err, 99)),
                   "rel_err_vs_setup_nu_max": float(np.max(err))},
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: a simulation runs on one GPU (served simulations are "
              "independent, one server per GPU; a single large grid would need y-slab sharding with halo "
              "exchanges, which this library does not implement). Requested --gpus %d." % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_02471_amd import lb, units, workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream(device=0)
    n, K, W, every = args.size, args.steps, args.warmup, args.sample_every
    cs, fd, prm = make_sims(lb, workloads, units, n, stream.cuda_stream)
    cap = (K + W) // every + 2
    cs.series_reserve(cap)
    fd.series_reserve(cap)
    # launch shapes of the plain steps chosen by the library's autotuner
    fd_tuned = fd.autotune(5)
    if args.fd_fused >= 0:
        fd.set_fd_fused(args.fd_fused)
    tuned = {"cs_threads": cs.autotune(10)[0], "fd_tile_rows": fd_tuned[1], "fd_tile_rows_later_stages": fd_tuned[2],
             "fd_fused_segment_rows": fd.fd_fused()}
    tuned["cs_nontemporal_stores"] = cs.cs_nontemporal()
    fused = fd.fd_fused() > 0
    run_cs = args.only in (None, "cs")
    run_fd = args.only in (None, "fd")

    # The two models advance in blocks of `every` steps: one sampled step
    # (diagnostics fused) and every - 1 plain steps, which the library
    # replays as captured HIP graphs.
    def chunks(n):
        return [every] * (n // every) + ([n % every] if n % every else [])

    for c in chunks(W):
        if run_cs:
            cs.step_sampled(c, every)
        if run_fd:
            fd.step_sampled(c, every)
    torch.cuda.synchronize()
    cs.series_read()
    fd.series_read()

    # K steps of each model, the CS steps first: the two simulations are
    # independent, and running each model's steps back to back keeps model
    # switches and timing markers out of the per-model times
    timed = chunks(K)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev[0].record(stream)
        if run_cs:
            for c in timed:
                cs.step_sampled(c, every)
        ev[1].record(stream)
        if run_fd:
            for c in timed:
                fd.step_sampled(c, every)
        ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cs_ms = ev[0].elapsed_time(ev[1]) / K
    fd_ms = ev[1].elapsed_time(ev[2]) / K
    ser_cs = cs.series_read()
    ser_fd = fd.series_read()
    assert np.all(np.isfinite(ser_cs)) and np.all(np.isfinite(ser_fd))

    nodes = n * n
    ms_per_step = wall * 1e3 / K
    bytes_cs = 2 * 9 * 4 * nodes                 # read + write 9 FP32 values per node
    # FD: three stage launches move 8 K s per step (8/3 K s per launch); the
    # fused step reads the state and its three moment planes once and writes
    # them once: (2 K s + 6 x 4) per step, one launch
    bytes_fd_stage = (8 * 16 * 4 * nodes) / 3.0 if not fused else (2 * 16 * 4 + 24) * nodes
    cs_gbs = bytes_cs / (cs_ms * 1e-3) / 1e9 if run_cs else 0.0
    fd_stage_ms = fd_ms / 3.0 if not fused else fd_ms
    fd_gbs = bytes_fd_stage / (fd_stage_ms * 1e-3) / 1e9 if run_fd else 0.0
    value = nodes / (ms_per_step * 1e-3) / 1e6

    line = {
        "metric": "MLUPS & % HBM peak (CS D2Q9, FD D2Q16); batched sims/s + p50/p99 latency",
        "value": round(value, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (closed-form Taylor-Green initial state; the paper uses no dataset)",
        "config": {
            "workload": "Taylor-Green vortex %dx%d periodic, u0=0.01, rho0=1: CS D2Q9 tau=0.6 (ds=dt=1) + "
                        "FD D2Q16 N=3 WENO-5/RK-3 at matched viscosity (tau_FD=%.5e, dt_FD=%.5e), FP32 storage "
                        "(shifted), FP64 diagnostics fused every %d steps; one update = one node advanced by "
                        "one CS step and one FD step" % (n, n, prm["tau_fd"], prm["dt_fd"], every),
            "grid": [n, n],
            "launch_shapes": tuned,
            "models": ["cs_d2q9" if run_cs else None, "fd_d2q16" if run_fd else None],
        },
        "cs_d2q9": {"ms_per_step": round(cs_ms, 5),
                    "mlups": round(nodes / (cs_ms * 1e-3) / 1e6, 1) if run_cs else None,
                    "achieved_gbs": round(cs_gbs, 1), "hbm_frac": round(cs_gbs / HBM_PEAK_GBS, 4),
                    "bytes_per_node_step": 72},
        "fd_d2q16": {"ms_per_step": round(fd_ms, 5),
                     "mlups": round(nodes / (fd_ms * 1e-3) / 1e6, 1) if run_fd else None,
                     "kernel": "fd_fused_step_kernel" if fused else "fd_stage_kernel (3 launches)",
                     "achieved_gbs": round(fd_gbs, 1), "hbm_frac": round(fd_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_node_step": 152 if fused else 512},
    }
    if run_fd:
        # The FD stage dominates the step.  Its two roofs, both against
        # published peaks: HBM (the stage-wise algorithmic bytes, 8 K s per
        # step = 8/3 K s per stage launch) and the FP32 vector ALU (the
        # algorithmic flops).  The binding roof is the one with the higher
        # fraction.  Launch duration: the FD step time over its three stage
        # launches (events on the launch stream around the FD steps).
        flops_launch = nodes * (16 * sum(FD16_FLOPS_NODE_POP) / 3.0 + FD16_FLOPS_NODE) * (3 if fused else 1)
        tflops = flops_launch / (fd_stage_ms * 1e-3) / 1e12
        hbm_frac = fd_gbs / HBM_PEAK_GBS
        alu_frac = tflops / VALU_PEAK_PUBLISHED_TFLOPS
        if hbm_frac >= alu_frac:
            roof = {"bound": "hbm", "achieved": round(fd_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_frac, 4)}
        else:
            roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": VALU_PEAK_PUBLISHED_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
        kname = "fd_fused_step_kernel" if fused else "fd_stage_kernel"
        if fused:
            rec = kernel_record(kname, n, {"segment_rows": fd.fd_fused()})
        else:
            rec = fd_stage_record(n, tuned["fd_tile_rows"], tuned["fd_tile_rows_later_stages"])
        line["roofline"] = dict(
            kernel=kname, **roof, traffic=rec["bytes_per_launch"] if rec else None,
            valu_issue=valu_issue(rec, fd_stage_ms),
            valu_issue_note="recorded SQ_INSTS_VALU and SQ_ACTIVE_INST_VALU2 per launch over 1024 SIMDs x the "
                            "quad-cycles at 2.4 GHz of the launch time measured here (null when the record does "
                            "not match this kernel's sources or launch shape)",
            bytes_per_launch=bytes_fd_stage, flops_per_launch=flops_launch,
            hbm_frac=round(hbm_frac, 4), alu_frac_published_peak=round(alu_frac, 4),
            alu_tflops=round(tflops, 2))
    else:
        line["roofline"] = {
            "kernel": "cs_step_vec_kernel", "bound": "hbm", "achieved": round(cs_gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(cs_gbs / HBM_PEAK_GBS, 4)}
        # workgroup size 0 is one 4-value chunk per thread: the row's chunk
        # count rounded up to whole waves, within [256, 1024]
        threads = tuned["cs_threads"] or min(1024, max(256, -(-(n // 4) // 64) * 64))
        rec = kernel_record("cs_step_vec_kernel", n, {"threads": threads, "nt": tuned["cs_nontemporal_stores"]})
        line["roofline"]["traffic"] = rec["bytes_per_launch"] if rec else None
        line["roofline"]["valu_issue"] = valu_issue(rec, cs_ms)
    if args.copy_calibration:
        src = torch.empty(bytes_cs // 8, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 20
        line["copy_calibration"] = {"bytes_moved": 2 * src.numel() * 4, "ms": round(ms, 5),
                                    "gbs": round(2 * src.numel() * 4 / (ms * 1e-3) / 1e9, 1)}
    line["host_boundary"] = host_boundary(
        lb, workloads, units, [(nm, sim, ms) for nm, sim, ms, on in
                               (("cs_d2q9", cs, cs_ms, run_cs), ("fd_d2q16", fd, fd_ms, run_fd)) if on], n, K)
    if args.only is None and not args.no_cache_free:
        cs.destroy()
        fd.destroy()
        line["cs_d2q9_4096"] = cache_free_cs(lb, workloads, stream)
        line["fd_d2q36"] = fd_d2q36(lb, workloads, units, stream)
        line["fd_d2q16_fused_vs_stages"] = fd_fused_compare(lb, workloads, units, stream)
    if args.serving_requests > 0:
        if args.only is not None or args.no_cache_free:
            cs.destroy()
            fd.destroy()
        line["serving"] = serving_bench(args.serving_requests, every, args.serving_batched_only,
                                        args.serving_node_limit, 1 if args.serving_policy == "shortest" else 0)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(every, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
