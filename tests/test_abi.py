"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/dmc.h declares, the ctypes structures match the C
layouts, and argument validation fails cleanly before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1206_3316_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(dmc_[a-z0-9_]+)\s*\(", text, flags=re.M))


def test_library_exports_every_declared_function():
    decl = declared_functions()
    assert len(decl) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB_PATH], capture_output=True, text=True, check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = sorted(decl - syms)
    assert not missing, missing
    assert decl == set(b.EXPORTS), sorted(decl ^ set(b.EXPORTS))


def test_library_loads_and_reports_version():
    L = b.lib()
    assert b"gfx950" in L.dmc_version()


@pytest.fixture(scope="module")
def layout_probe(tmp_path_factory):
    src = tmp_path_factory.mktemp("abi") / "probe.c"
    exe = str(src.with_suffix(""))
    structs = {
        "dmc_branch": ["n_bins", "omega", "domega", "dos", "vg", "tau", "degeneracy"],
        "dmc_wall": ["type", "temperature", "specularity"],
        "dmc_geometry_desc": ["kind", "length", "radius", "wall"],
        "dmc_source": ["kind", "dT", "radius", "gradient"],
        "dmc_tally_desc": ["n_bins", "n_batches", "kmax", "n_hj", "grid", "grid_lo", "grid_hi", "first_event",
                           "region", "region_c", "region_radius", "region_z"],
        "dmc_run_opts": ["precision", "form", "stream", "block", "chunk", "refill_min", "lds_tally", "grid_blocks",
                         "workspace", "workspace_bytes", "nscat_out", "prio_flights", "nscat_out_len"],
        "dmc_job": ["material", "geometry", "source", "tally", "n_particles", "seed", "times", "n_times",
                    "first_particle"],
        "dmc_stats": ["particles", "scatters", "boundary", "iterations", "capped", "kernel_ms", "flights"],
        "dmc_server_opts": ["memory_budget", "max_active", "epoch_flights", "drain_flights", "class_epochs", "run"],
        "dmc_trunc_opts": ["n_pilot", "k_pilot", "bias_fraction"],
        "dmc_trunc_plan": ["kmax", "k_uncertain", "fit_ok", "n_fit", "decay", "amplitude", "bias_bound", "kappa_se",
                           "kappa_pilot", "n_pilot"],
        "dmc_tune_trial": ["block", "chunk", "refill_min", "lds_tally", "pilot", "ms", "flights_per_s"],
        "dmc_tune_opts": ["sample_flights", "trial_cap", "use_cache", "trials", "max_trials", "n_trials",
                          "from_cache"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for s, fields in structs.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("  return 0; }")
    src.write_text("\n".join(lines))
    subprocess.check_call(["gcc", "-std=c11", "-o", exe, str(src)])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return structs, out


def test_ctypes_structures_match_c_layout(layout_probe):
    structs, out = layout_probe
    got = {}
    for ln in out.splitlines():
        parts = ln.split()
        got[(parts[0], parts[1])] = int(parts[2])
    for s, fields in structs.items():
        cls = getattr(b, s)
        assert C.sizeof(cls) == got[(s, "size")], s
        for f in fields:
            assert getattr(cls, f).offset == got[(s, f)], (s, f)


def test_invalid_arguments_fail_cleanly_without_a_device():
    """Validation happens before any HIP call and reports a message."""
    out = C.c_void_p(123)
    rc = b.lib().dmc_material_create(None, 0, 300.0, 0.0, C.byref(out))
    assert rc == b.DMC_E_INVALID and out.value is None
    assert b"branch" in b.lib().dmc_last_error()
    br = (b.dmc_branch * 1)()
    om = np.array([1e13, -1.0])
    ones = np.ones(2)
    p = lambda a: a.ctypes.data_as(b.f64p)
    br[0] = b.dmc_branch(2, p(om), p(ones), p(ones), p(ones), p(ones), 1.0)
    rc = b.lib().dmc_material_create(br, 1, 300.0, 0.0, C.byref(out))
    assert rc == b.DMC_E_INVALID and b"non-physical" in b.lib().dmc_last_error()
    om[1] = 2e13
    for g in (1.0, -1.0, float("nan")):
        rc = b.lib().dmc_material_create(br, 1, 300.0, g, C.byref(out))
        assert rc == b.DMC_E_INVALID and b"scatter_g" in b.lib().dmc_last_error()
    d = b.dmc_geometry_desc()
    d.kind = 7
    rc = b.lib().dmc_geometry_create(C.byref(d), C.byref(out))
    assert rc == b.DMC_E_INVALID
    d.kind = 2
    d.length = 1e-7
    d.radius = 0.6e-7
    d.wall[0] = b.dmc_wall(1, 0.0, 0.0)
    rc = b.lib().dmc_geometry_create(C.byref(d), C.byref(out))
    assert rc == b.DMC_E_INVALID and b"radius" in b.lib().dmc_last_error()
    o = b.dmc_run_opts()
    b.lib().dmc_run_opts_default(C.byref(o))
    assert o.precision == 1 and o.form == 1 and o.lds_tally == 1


def test_geometry_handles_without_device():
    """Geometry creation is pure host work."""
    import dmc_inputs as di
    g = b.Geometry(di.gray_slab().geometry)
    assert g.handle.value
    del g


def test_autotune_validates_before_device_work():
    best = b.dmc_run_opts()
    assert b.lib().dmc_autotune(None, 0, None, None, C.byref(best)) == b.DMC_E_INVALID
    assert b.lib().dmc_autotune(None, 1, None, None, None) == b.DMC_E_INVALID


def test_truncation_planning_validates_before_device_work():
    j = b.dmc_job()
    j.source.kind = 0  # wall sources: truncation planning needs the gradient source
    j.n_particles = 100
    out = b.dmc_trunc_plan()
    assert b.lib().dmc_plan_truncation(C.byref(j), None, None, C.byref(out)) == b.DMC_E_INVALID
    assert b"gradient" in b.lib().dmc_last_error()
    assert b.lib().dmc_plan_truncation(None, None, None, None) == b.DMC_E_INVALID


def test_debug_philox_rejects_null():
    rc = b.lib().dmc_debug_philox(1, None, None, None, None, 4)
    assert rc == b.DMC_E_INVALID


def test_binding_refuses_host_buffers_for_device_outputs():
    """A workspace or scattering-count buffer in host memory (or a strided one)
    is refused by the binding before any library call: the kernels write to them
    from the device."""
    torch = pytest.importorskip("torch")
    import dmc_inputs as di
    job = di.gray_slab()
    job.n_particles = 100
    for kw in ({"workspace": torch.zeros(1 << 20, dtype=torch.uint8)},
               {"nscat_out": torch.zeros(100, dtype=torch.int32)}):
        with pytest.raises(ValueError):
            b.simulate([job], **kw)
        with pytest.raises(ValueError):
            b.simulate_one(job, **kw)
    strided = torch.zeros((100, 2), dtype=torch.int32)[:, 0]
    with pytest.raises(ValueError):
        b.simulate([job], nscat_out=strided)
