"""CPU checks of the benchmark driver's contract (no device needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    line = [l for l in r.stdout.splitlines() if l.strip()][-1]
    assert "one GPU only" in json.loads(line)["error"]


def test_kernel_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    """The traffic figure stays valid across comment edits and is dropped on any
    code change: the hash covers the device code with comments and spacing removed."""
    csrc = tmp_path / "paper_1206_3316_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "dmc_internal.h").write_text("struct A { int x; }; // a note\n")
    (csrc / "dmc_kernels.hip").write_text("int f(int a) { return a + 1; } /* block\n comment */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sha1()
    (csrc / "dmc_kernels.hip").write_text("// new comment\nint  f(int a)\n{\n    return a + 1;\n}\n")
    assert bench.kernel_sha1() == h0
    (csrc / "dmc_kernels.hip").write_text("int f(int a) { return a + 2; }\n")
    assert bench.kernel_sha1() != h0


def test_traffic_figure_names_a_kernel_hash():
    t = bench.TRAFFIC
    assert len(t["kernel_sha1"]) == 40 and t["bytes"] > 0
    assert bench.OPS_PER_FLIGHT > 0
