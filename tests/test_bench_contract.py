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


NOMINAL = {"fma": 1.0, "philox_uniform_key": 43.0, "philox_lane_key": 61.0, "log": 2.0, "sin": 2.0, "cos": 2.0,
           "sqrt": 2.0, "rcp": 1.0, "f64_add": 1.0}


def test_algorithmic_counts_are_itemised():
    """Every item of the per-flight counts is positive and named; with the
    nominal costs the slab flight is the 84 slots itemised in the design notes."""
    for items in (bench.slab_items(NOMINAL), bench.half_items(NOMINAL)):
        assert all(isinstance(k, str) and v > 0 for k, v in items)
    assert sum(v for _, v in bench.slab_items(NOMINAL)) == 84
    u = bench.grad_unit_costs(NOMINAL)
    assert u["segment_pore"] > u["segment_film"] > 0 and u["flight"] > 43


def test_gradient_roofline_splits_events_by_kind():
    """grad_roofline derives periodic crossings (segments - flights) and surface
    interactions (boundary - periodic) per job and prices each at its unit cost."""
    from types import SimpleNamespace as NS
    jobs = [NS(geometry=NS(kind="film_x")), NS(geometry=NS(kind="pore_cell_xz"))]
    st = [NS(flights=100, iterations=100, scatters=80, boundary=20),
          NS(flights=50, iterations=70, scatters=40, boundary=30)]
    r = bench.grad_roofline(jobs, st, 1.0, NOMINAL)
    u = bench.grad_unit_costs(NOMINAL)
    ev = r["ops_by_event"]
    assert ev["periodic"] == 20 * u["periodic"]
    assert ev["hit"] == 20 * u["wall_hit"] + 10 * u["pore_hit"]
    assert ev["segment"] == 100 * u["segment_film"] + 70 * u["segment_pore"]
    assert ev["flight"] == 150 * u["flight"] and ev["scatter"] == 120 * u["scatter"]
    assert abs(r["frac"] - sum(ev.values()) / 1e-3 / bench.PEAK_LANE_OPS) < 1e-12


def test_host_cpu_names_a_model():
    c = bench.host_cpu()
    assert c["model"] and c["logical_cpus"] >= 1
