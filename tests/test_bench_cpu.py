"""Host logic of bench.py (no GPU): the one-GPU contract and the reporting
of measured kernel traffic and VALU issue only while the kernel's sources and
launch shape are those the counters were taken on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    bench = load_bench()
    csrc = os.path.join(ROOT, "paper_1904_02471_amd", "csrc")
    files = ["lb_fd_impl.h", "lb_fd.hip"]
    inst = {"stage1_rows8": {"bytes": 9000, "valu_insts": 1.0e8, "valu_pairs": 2.4e7},
            "stage23_rows4": {"bytes": 13000, "valu_insts": 1.3e8, "valu_pairs": 3.3e7},
            "stage1_rows4": {"bytes": 9600}}
    record = {"fd_stage_kernel": {"grid": [64, 64], "sources": files, "sources_sha256": bench.source_digest(files),
                                  "instances": inst},
              "fd_fused_step_kernel": {"grid": [64, 64], "sources": files, "sources_sha256": bench.source_digest(files),
                                       "segment_rows": 32, "bytes_per_launch": 4321}}
    pkg = tmp_path / "paper_1904_02471_amd"
    (pkg / "csrc").mkdir(parents=True)
    for f in files:
        (pkg / "csrc" / f).write_bytes(open(os.path.join(csrc, f), "rb").read())
    (pkg / "kernel_traffic.json").write_text(json.dumps(record))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # one first-stage launch and two later ones per step
    rec = bench.fd_stage_record(64, 8, 4)
    assert rec["bytes_per_launch"] == (9000 + 2 * 13000) / 3.0
    assert rec["valu_insts_per_launch"] == (1.0e8 + 2 * 1.3e8) / 3.0
    assert rec["valu_pairs_per_launch"] == (2.4e7 + 2 * 3.3e7) / 3.0
    # the VALU issue of a launch of 1.2e8 wave instructions, 3e7 of the
    # quad-cycles issuing two, over the 1024 SIMDs x 0.6e9 quad-cycles per
    # second x 0.25 ms
    rec = {"valu_insts_per_launch": 1.2e8, "valu_pairs_per_launch": 3.0e7}
    quads = 1024 * 0.6e9 * 0.25e-3
    issue = bench.valu_issue(rec, 0.25)
    assert issue["insts_per_quad_cycle"] == round(1.2e8 / quads, 4)
    assert issue["busy_frac"] == round((1.2e8 - 3.0e7) / quads, 4)
    assert issue["paired_share"] == 0.5
    del rec["valu_pairs_per_launch"]
    assert set(bench.valu_issue(rec, 0.25)) == {"insts_per_quad_cycle"}
    assert bench.valu_issue(None, 0.25) is None
    # an instance recorded without instruction counts gives bytes only
    rec = bench.fd_stage_record(64, 4, 4)
    assert rec == {"bytes_per_launch": (9600 + 2 * 13000) / 3.0}
    assert bench.fd_stage_record(64, 8, 8) is None  # no record of that later-stage instance
    assert bench.fd_stage_record(128, 8, 4) is None  # another workload
    assert bench.kernel_record("fd_fused_step_kernel", 64, {"segment_rows": 32})["bytes_per_launch"] == 4321
    assert bench.kernel_record("fd_fused_step_kernel", 64, {"segment_rows": 64}) is None  # another launch shape
    assert bench.kernel_record("cs_step_vec_kernel", 64) is None  # no record
    with open(pkg / "csrc" / "lb_fd.hip", "ab") as fh:  # the kernel changed since the counters
        fh.write(b"\n// edited\n")
    assert bench.fd_stage_record(64, 8, 4) is None
    assert bench.kernel_record("fd_fused_step_kernel", 64) is None
