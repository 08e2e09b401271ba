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
          "tri_lookups": 20, "tri_pairs": 7}


def test_sweep_bytes_model(bench):
    b = bench.sweep_bytes(CENSUS, [CENSUS, CENSUS], tables=False)
    assert b["sweep3_fwd_count"] == 16 * 10 + 12 * 100
    assert b["sweep3_bwd_count"] == 16 * 10 + 12 * 90
    assert b["sweep3_tri_count"] == 16 * 5 + 12 * 50 + 48 * 20 + 96 * 7
    assert b["sweep3_tri_weight"] == 2 * (16 * 5 + 20 * 50 + 24 * 20 + 72 * 7)
    t = bench.sweep_bytes(CENSUS, [], tables=True)
    assert t["sweep3_fwd_count"] == 344 * 10 and t["sweep3_bwd_count"] == 336 * 10


def test_dominant_kernel_is_the_one_with_most_time_alone(bench):
    # in the timed (concurrent) steps the forward kernel looks longest, but
    # alone the triangle kernel takes the most time: it is the dominant one
    kern = {"sweep3_fwd_weight": (240.0, 4), "sweep3_tri_weight": (200.0, 4), "sweep3_tri_count": (140.0, 1)}
    alone = {"sweep3_fwd_weight": (70.0, 4), "sweep3_tri_weight": (190.0, 4), "sweep3_tri_count": (135.0, 1)}
    crit = {"sweep3_fwd_weight": (190.0, 3)}
    r = bench.sweep_roofline(CENSUS, [CENSUS] * 4, kern, crit, alone, 1, tables=True)
    assert r["kernel"] == "sweep3_tri_weight"
    per = r["sweep_kernels"]["sweep3_tri_weight"]
    assert per["avg_launch_ms"] == pytest.approx(50.0)
    assert r["achieved"] == pytest.approx(per["algorithmic_bytes_per_launch"] / 0.050 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
