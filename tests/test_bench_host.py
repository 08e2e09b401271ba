"""Host-side pieces of bench.py (no GPU): the traffic-record hash, the
algorithmic byte model and the choice of the dominant kernel."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as b
    return b


def test_code_only_drops_comments_keeps_literals(bench):
    src = 'int a = 1; // note\n/* block\n comment */ const char *s = "//not a comment"; char c = \'/\';\n\n  int  d;'
    assert bench._code_only(src) == 'int a = 1; const char *s = "//not a comment"; char c = \'/\'; int d;'
    # a change of comments or spacing keeps the hash of the code
    assert bench._code_only(src) == bench._code_only(src.replace("// note", "// other note").replace("  ", " "))
    assert bench._code_only(src) != bench._code_only(src.replace("a = 1", "a = 2"))


CENSUS = {"anchors": 10, "fwd_entries": 100, "bwd_entries": 90, "tri_anchors": 5, "tri_entries": 50,
          "tri_lookups": 20, "tri_pairs": 7, "tri_probes": 33}


def test_sweep_bytes_model(bench):
    """16 B per anchor, 12 B per scanned entry (20 with the weight), 8 B per
    probe; the tables of the exact 2-node/star counts do not change the
    algorithmic bytes (the scans they replace)."""
    b = bench.sweep_bytes(CENSUS, [CENSUS, CENSUS])
    assert b["sweep3_fwd_count"] == 16 * 10 + 12 * 100
    assert b["sweep3_bwd_count"] == 16 * 10 + 12 * 90
    assert b["sweep3_tri_count"] == 16 * 5 + 12 * 50 + 8 * 33
    assert b["sweep3_tri_weight"] == 2 * (16 * 5 + 20 * 50 + 8 * 33)
    assert b["sweep3_fwd_weight"] == 2 * (16 * 10 + 20 * 100)
    assert "tri_static_weight" not in b


def test_static_triangle_bytes_model(bench):
    """Weighted triangles over static triangles: 48 B per unit, 48 B per
    driver entry, 24 B per (first, last) pair, summed over the estimate
    settings; absent when a setting has no static census."""
    st = {"triangles": 9, "units": 3, "tasks": 40, "drivers": 11, "steps": 5, "combos": 70}
    ests = [dict(CENSUS, static=st), dict(CENSUS, static=dict(st, units=1, drivers=2, combos=4))]
    b = bench.sweep_bytes(CENSUS, ests)
    assert b["tri_static_weight"] == (48 * 3 + 48 * 11 + 24 * 70) + (48 * 1 + 48 * 2 + 24 * 4)
    b = bench.sweep_bytes(CENSUS, [dict(CENSUS, static=st), dict(CENSUS, static=None)])
    assert "tri_static_weight" not in b


def test_dominant_kernel_and_counter_based_fraction(bench, monkeypatch):
    # in the timed (concurrent) steps the forward kernel looks longest, but
    # alone the triangle kernel takes the most time: it is the dominant one
    kern = {"sweep3_fwd_weight": (240.0, 4), "sweep3_tri_weight": (200.0, 4), "sweep3_tri_count": (140.0, 1)}
    alone = {"sweep3_fwd_weight": (70.0, 4), "sweep3_tri_weight": (190.0, 4), "sweep3_tri_count": (135.0, 1)}
    crit = {"sweep3_fwd_weight": (190.0, 3)}
    # with a valid counter record, frac is its bytes per launch over the launch time
    monkeypatch.setattr(bench, "traffic_record", lambda k: 4.0e9 if k == "sweep3_tri_weight" else None)
    r = bench.sweep_roofline(CENSUS, [CENSUS] * 4, kern, crit, alone, 1)
    assert r["kernel"] == "sweep3_tri_weight"
    per = r["sweep_kernels"]["sweep3_tri_weight"]
    assert per["avg_launch_ms"] == pytest.approx(50.0)
    assert r["traffic"] == 4.0e9
    assert r["achieved"] == pytest.approx(4.0e9 / 0.050 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["algorithmic"]["bytes_per_launch"] == pytest.approx(per["algorithmic_bytes_per_launch"])
    assert r["algorithmic"]["GBs"] == pytest.approx(per["algorithmic_bytes_per_launch"] / 0.050 / 1e9)
    # a stale record: traffic null, frac from the algorithmic bytes, and said so
    monkeypatch.setattr(bench, "traffic_record", lambda k: None)
    r = bench.sweep_roofline(CENSUS, [CENSUS] * 4, kern, crit, alone, 1)
    assert r["traffic"] is None and "stale" in r["frac_basis"]
    assert r["achieved"] == pytest.approx(per["algorithmic_bytes_per_launch"] / 0.050 / 1e9)


def test_pmc_and_trace_summaries(bench, tmp_path, monkeypatch):
    """The traffic record and the kernel-trace summary are computed from
    rocprofv3's csv files: counters scaled by the copy calibration, the
    sweep kernels' timed-step dispatches only."""
    def write(folder, name, header, rows):
        d = tmp_path / folder / "host" / "123"
        d.mkdir(parents=True, exist_ok=True)
        with open(d / f"run_{name}", "w") as f:
            f.write(",".join(header) + "\n")
            for r in rows:
                f.write(",".join(str(x) for x in r) + "\n")
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    tri = '"void (anonymous namespace)::k_sweep3<1, true, 8u>(DevGraph, sweepdev::SweepArgs)"'
    write("f", "counter_collection.csv", hdr, [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0],
                                              [2, tri, "FETCH_SIZE", 100.0], [3, tri, "FETCH_SIZE", 300.0]])
    write("w", "counter_collection.csv", hdr, [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0],
                                              [2, tri, "WRITE_SIZE", 10.0], [3, tri, "WRITE_SIZE", 30.0]])
    monkeypatch.setattr(bench, "traffic_file", lambda k: str(tmp_path / f"{k}.json"))
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"))
    import json
    rec = json.load(open(tmp_path / "sweep3_tri_weight.json"))
    assert rec["dispatches_averaged"] == 2
    assert rec["traffic_bytes_per_launch"] == pytest.approx((200.0 * 2 + 20.0) * 1024)
    assert rec["kernel_src_sha256"] == bench.kernel_src_sha()


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_serve_merge_pairs_phases(bench):
    """Serving lines from separate server and one-at-a-time runs join per
    arrival rate; differing results are counted (counts exactly, estimates
    beyond 1e-12 relative) and the value is the server's throughput at the
    highest rate meeting the p99 target."""
    def ph(qps, phase, p99, eps, results):
        return {"qps": qps, "phase": phase, "queries": 3, "edges": 30, "p50_ms": 1.0, "p99_ms": p99,
                "wall_s": 2.0, "edges_per_s": eps, "results": results}
    phases = [ph(2.0, "server", 100.0, 20.0, ["7", 1.5, 2.0]),
              ph(2.0, "one_at_a_time", 600.0, 10.0, ["7", 1.5, 2.0 * (1 + 1e-9)]),
              ph(4.0, "server", 900.0, 40.0, ["8", 1.0, 3.0]),
              ph(4.0, "one_at_a_time", 2000.0, 15.0, ["9", 1.0, 3.0])]
    out = bench.serve_merge(phases, {"workload": "w"}, 500.0)
    sw = {s["qps"]: s for s in out["sweep"]}
    assert sw[2.0]["results_differing_from_one_at_a_time"] == 1
    assert sw[4.0]["results_differing_from_one_at_a_time"] == 1
    assert sw[2.0]["server_meets_p99_target"] and not sw[2.0]["one_at_a_time_meets_p99_target"]
    assert not sw[4.0]["server_meets_p99_target"]
    assert out["value"] == 20.0 and out["config"]["value_at_qps"] == 2.0
    assert abs(sw[2.0]["server_over_one_at_a_time_throughput"] - 2.0) < 1e-12
