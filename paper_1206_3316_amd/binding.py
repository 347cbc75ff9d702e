"""ctypes binding of include/dmc.h (argument marshalling only).

Every function named ``dmc_*`` here has the name and argument order of the C
entry point it calls; the classes below only convert the seeded problem
descriptions of ``dmc_inputs`` into the C structures and keep handles alive.
All simulation work runs in the HIP kernels of ``libdmc.so``.  PyTorch is
used only to provide device memory (the workspace) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmc.so")

DMC_OK, DMC_E_INVALID, DMC_E_NOMEM, DMC_E_DEVICE, DMC_E_UNSUPPORTED, DMC_E_BUSY = 0, -1, -2, -3, -4, -5
GEOM = {"slab_z": 0, "film_x": 1, "pore_cell_xz": 2, "halfspace_z": 3}
WALL = {"isothermal": 0, "adiabatic": 1, "periodic": 2}
SRC = {"walls": 0, "gaussian": 1, "gradient": 2}
PREC = {"fp64": 0, "fp32": 1}
FORM = {"plain": 0, "persistent": 1}
(Q_T, Q_TLOC, Q_FLUX, Q_KAPPA, Q_HJ, Q_SNAPSHOT, Q_SNAPSHOT_SUM, Q_RAW, Q_REGION_T, Q_REGION_QZ,
 Q_FIELD_T, Q_FIELD_QZ) = range(12)
TABLE_GAIN, TABLE_INIT, TABLE_FLUX = 0, 1, 2

f64p = C.POINTER(C.c_double)
u32p = C.POINTER(C.c_uint32)


class dmc_branch(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("omega", f64p), ("domega", f64p), ("dos", f64p), ("vg", f64p),
                ("tau", f64p), ("degeneracy", C.c_double)]


class dmc_wall(C.Structure):
    _fields_ = [("type", C.c_int32), ("temperature", C.c_double), ("specularity", C.c_double)]


class dmc_geometry_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("length", C.c_double), ("radius", C.c_double), ("wall", dmc_wall * 2)]


class dmc_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dT", C.c_double), ("radius", C.c_double), ("gradient", C.c_double)]


class dmc_tally_desc(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("n_batches", C.c_int32), ("kmax", C.c_int32), ("n_hj", C.c_int32),
                ("grid", C.c_int32 * 3), ("grid_lo", C.c_double * 3), ("grid_hi", C.c_double * 3),
                ("first_event", C.c_int32), ("region", C.c_int32), ("region_c", C.c_double * 2),
                ("region_radius", C.c_double), ("region_z", C.c_double * 2)]


class dmc_run_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("form", C.c_int32), ("stream", C.c_void_p), ("block", C.c_int32),
                ("chunk", C.c_int32), ("refill_min", C.c_int32), ("lds_tally", C.c_int32),
                ("grid_blocks", C.c_int32), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("nscat_out", C.c_void_p), ("prio_flights", C.c_int32), ("pad0", C.c_int32),
                ("nscat_out_len", C.c_uint64)]


class dmc_job(C.Structure):
    _fields_ = [("material", C.c_void_p), ("geometry", C.c_void_p), ("source", dmc_source),
                ("tally", dmc_tally_desc), ("n_particles", C.c_uint64), ("seed", C.c_uint64),
                ("times", f64p), ("n_times", C.c_int32), ("pad0", C.c_int32), ("first_particle", C.c_uint64)]


class dmc_stats(C.Structure):
    _fields_ = [("particles", C.c_uint64), ("scatters", C.c_uint64), ("boundary", C.c_uint64),
                ("iterations", C.c_uint64), ("capped", C.c_uint64), ("kernel_ms", C.c_double),
                ("flights", C.c_uint64)]


class dmc_tune_trial(C.Structure):
    _fields_ = [("block", C.c_int32), ("chunk", C.c_int32), ("refill_min", C.c_int32), ("lds_tally", C.c_int32),
                ("pilot", C.c_int32), ("pad0", C.c_int32), ("ms", C.c_double), ("flights_per_s", C.c_double)]


class dmc_tune_opts(C.Structure):
    _fields_ = [("sample_flights", C.c_uint64), ("trial_cap", C.c_uint32), ("use_cache", C.c_int32),
                ("trials", C.POINTER(dmc_tune_trial)), ("max_trials", C.c_int32), ("n_trials", C.c_int32),
                ("from_cache", C.c_int32)]


class dmc_trunc_opts(C.Structure):
    _fields_ = [("n_pilot", C.c_uint64), ("k_pilot", C.c_int32), ("pad0", C.c_int32), ("bias_fraction", C.c_double)]


class dmc_trunc_plan(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("k_uncertain", C.c_int32), ("fit_ok", C.c_int32), ("n_fit", C.c_int32),
                ("decay", C.c_double), ("amplitude", C.c_double), ("bias_bound", C.c_double),
                ("kappa_se", C.c_double), ("kappa_pilot", C.c_double), ("n_pilot", C.c_uint64)]


class dmc_server_opts(C.Structure):
    _fields_ = [("memory_budget", C.c_size_t), ("max_active", C.c_int32), ("epoch_flights", C.c_uint64),
                ("drain_flights", C.c_uint32), ("class_epochs", C.c_int32), ("run", dmc_run_opts)]


_SIGS = {
    "dmc_last_error": ([], C.c_char_p),
    "dmc_version": ([], C.c_char_p),
    "dmc_material_create": ([C.POINTER(dmc_branch), C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_void_p)],
                            C.c_int32),
    "dmc_material_destroy": ([C.c_void_p], C.c_int32),
    "dmc_material_info": ([C.c_void_p, C.POINTER(C.c_int32), f64p], C.c_int32),
    "dmc_geometry_create": ([C.POINTER(dmc_geometry_desc), C.POINTER(C.c_void_p)], C.c_int32),
    "dmc_geometry_destroy": ([C.c_void_p], C.c_int32),
    "dmc_run_opts_default": ([C.POINTER(dmc_run_opts)], None),
    "dmc_workspace_size": ([C.POINTER(dmc_job), C.c_int32, C.POINTER(dmc_run_opts), C.POINTER(C.c_size_t)],
                           C.c_int32),
    "dmc_simulate": ([C.c_void_p, C.c_void_p, C.POINTER(dmc_source), C.c_uint64, C.c_uint64,
                      C.POINTER(dmc_tally_desc), f64p, C.c_int32, C.POINTER(dmc_run_opts), C.POINTER(C.c_void_p)],
                     C.c_int32),
    "dmc_simulate_batch": ([C.POINTER(dmc_job), C.c_int32, C.POINTER(dmc_run_opts), C.POINTER(C.c_void_p)],
                           C.c_int32),
    "dmc_simulate_batch_noalloc": ([C.POINTER(dmc_job), C.c_int32, C.POINTER(dmc_run_opts), C.c_void_p, C.c_size_t,
                                    C.c_void_p, C.POINTER(C.c_size_t)], C.c_int32),
    "dmc_autotune": ([C.POINTER(dmc_job), C.c_int32, C.POINTER(dmc_run_opts), C.POINTER(dmc_tune_opts),
                      C.POINTER(dmc_run_opts)], C.c_int32),
    "dmc_plan_truncation": ([C.POINTER(dmc_job), C.POINTER(dmc_run_opts), C.POINTER(dmc_trunc_opts),
                             C.POINTER(dmc_trunc_plan)], C.c_int32),
    "dmc_tally_read": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, f64p, f64p, C.c_size_t], C.c_int32),
    "dmc_tally_raw_size": ([C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)], C.c_int32),
    "dmc_result_stats": ([C.c_void_p, C.c_int32, C.POINTER(dmc_stats)], C.c_int32),
    "dmc_result_destroy": ([C.c_void_p], C.c_int32),
    "dmc_server_create": ([C.c_void_p, C.POINTER(dmc_server_opts), C.POINTER(C.c_void_p)], C.c_int32),
    "dmc_server_submit": ([C.c_void_p, C.POINTER(dmc_job), C.POINTER(C.c_uint64)], C.c_int32),
    "dmc_server_step": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int32),
    "dmc_server_poll": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)], C.c_int32),
    "dmc_server_wait": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)], C.c_int32),
    "dmc_server_collect": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_void_p)], C.c_int32),
    "dmc_server_load": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int32),
    "dmc_server_totals": ([C.c_void_p, C.POINTER(dmc_stats)], C.c_int32),
    "dmc_server_destroy": ([C.c_void_p], C.c_int32),
    "dmc_debug_philox": ([C.c_uint64, C.POINTER(C.c_uint64), u32p, u32p, u32p, C.c_size_t], C.c_int32),
    "dmc_debug_alias": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32), u32p, u32p, C.c_size_t], C.c_int32),
    "dmc_debug_alias_draw": ([C.c_void_p, C.c_int32, u32p, u32p, C.c_size_t], C.c_int32),
    "dmc_debug_fp64_math": ([f64p, f64p, f64p, f64p, C.c_size_t], C.c_int32),
    "dmc_debug_op_cost": ([C.c_int32, C.c_uint32, C.c_int32, f64p, C.POINTER(C.c_uint64)], C.c_int32),
}

EXPORTS = tuple(_SIGS)

_lib = None


class DmcError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def lib() -> C.CDLL:
    """Load libdmc.so.  Raises if it was not built: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_1206_3316_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(fn: str, rc: int):
    if rc != DMC_OK:
        raise DmcError(fn, rc, lib().dmc_last_error().decode())


def _call(name, *args):
    rc = getattr(lib(), name)(*args)
    check(name, rc)
    return rc


# thin wrappers with the C names -------------------------------------------

def dmc_material_create(branches, n_branches, T_eq, scatter_g, out):
    return _call("dmc_material_create", branches, n_branches, T_eq, scatter_g, out)


def dmc_material_destroy(m):
    return _call("dmc_material_destroy", m)


def dmc_material_info(m, n_states, sums):
    return _call("dmc_material_info", m, n_states, sums)


def dmc_geometry_create(desc, out):
    return _call("dmc_geometry_create", desc, out)


def dmc_geometry_destroy(g):
    return _call("dmc_geometry_destroy", g)


def dmc_run_opts_default(opts):
    lib().dmc_run_opts_default(opts)


def dmc_workspace_size(jobs, n_jobs, opts, nbytes):
    return _call("dmc_workspace_size", jobs, n_jobs, opts, nbytes)


def dmc_simulate(material, geometry, source, n_particles, seed, tally, times, n_times, opts, out):
    return _call("dmc_simulate", material, geometry, source, n_particles, seed, tally, times, n_times, opts, out)


def dmc_simulate_batch(jobs, n_jobs, opts, out):
    return _call("dmc_simulate_batch", jobs, n_jobs, opts, out)


def dmc_simulate_batch_noalloc(jobs, n_jobs, opts, raw_out, raw_len, counters_out, raw_offsets):
    return _call("dmc_simulate_batch_noalloc", jobs, n_jobs, opts, raw_out, raw_len, counters_out, raw_offsets)


def dmc_autotune(jobs, n_jobs, base, tune, best):
    return _call("dmc_autotune", jobs, n_jobs, base, tune, best)


def dmc_plan_truncation(job, opts, t, out):
    return _call("dmc_plan_truncation", job, opts, t, out)


def dmc_tally_read(res, job, quantity, time_index, mean, se, n):
    return _call("dmc_tally_read", res, job, quantity, time_index, mean, se, n)


def dmc_tally_raw_size(res, job, n):
    return _call("dmc_tally_raw_size", res, job, n)


def dmc_result_stats(res, job, out):
    return _call("dmc_result_stats", res, job, out)


def dmc_result_destroy(res):
    return _call("dmc_result_destroy", res)


def dmc_server_create(material, opts, out):
    return _call("dmc_server_create", material, opts, out)


def dmc_server_submit(server, job, ticket):
    return _call("dmc_server_submit", server, job, ticket)


def dmc_server_step(server, n_done):
    return _call("dmc_server_step", server, n_done)


def dmc_server_poll(server, ticket, done):
    return _call("dmc_server_poll", server, ticket, done)


def dmc_server_wait(server, ticket, n_epochs):
    return _call("dmc_server_wait", server, ticket, n_epochs)


def dmc_server_collect(server, ticket, out):
    return _call("dmc_server_collect", server, ticket, out)


def dmc_server_load(server, queued, running):
    return _call("dmc_server_load", server, queued, running)


def dmc_server_totals(server, out):
    return _call("dmc_server_totals", server, out)


def dmc_server_destroy(server):
    return _call("dmc_server_destroy", server)


def dmc_debug_philox(seed, pid, k, tag, out, n):
    return _call("dmc_debug_philox", seed, pid, k, tag, out, n)


def dmc_debug_alias(m, which, bits, thresh, alias, n):
    return _call("dmc_debug_alias", m, which, bits, thresh, alias, n)


def dmc_debug_alias_draw(m, which, words, states, n):
    return _call("dmc_debug_alias_draw", m, which, words, states, n)


# marshalling helpers --------------------------------------------------------

def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Material:
    """Owns a dmc_material built from a ``dmc_inputs.Material``."""

    def __init__(self, material):
        self.src = material
        self._keep = []
        brs = (dmc_branch * len(material.branches))()
        for i, b in enumerate(material.branches):
            arrs = [np.ascontiguousarray(getattr(b, n), np.float64) for n in ("omega", "domega", "dos", "vg", "tau")]
            self._keep += arrs
            brs[i] = dmc_branch(arrs[0].shape[0], *[_ptr(a, C.c_double) for a in arrs], float(b.degeneracy))
        h = C.c_void_p()
        dmc_material_create(brs, len(material.branches), float(material.T_eq),
                            float(getattr(material, "scatter_g", 0.0)), C.byref(h))
        self.handle = h

    def info(self):
        n = C.c_int32()
        sums = np.zeros(3)
        dmc_material_info(self.handle, C.byref(n), _ptr(sums, C.c_double))
        return int(n.value), sums

    def alias_table(self, which: int):
        bits = C.c_int32()
        dmc_debug_alias(self.handle, which, C.byref(bits), None, None, 0)
        n = 1 << bits.value
        th = np.zeros(n, np.uint32)
        al = np.zeros(n, np.uint32)
        dmc_debug_alias(self.handle, which, C.byref(bits), _ptr(th, C.c_uint32), _ptr(al, C.c_uint32), n)
        return {"bits": bits.value, "thresh": th, "alias": al}

    def alias_draw(self, which: int, words: np.ndarray) -> np.ndarray:
        w = np.ascontiguousarray(words, np.uint32)
        out = np.zeros(w.shape[0], np.uint32)
        dmc_debug_alias_draw(self.handle, which, _ptr(w, C.c_uint32), _ptr(out, C.c_uint32), w.shape[0])
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.dmc_material_destroy(self.handle)
        except Exception:
            pass


class Geometry:
    def __init__(self, geometry):
        d = dmc_geometry_desc()
        d.kind = GEOM[geometry.kind]
        d.length = float(geometry.length)
        d.radius = float(geometry.radius)
        walls = list(geometry.walls)
        while len(walls) < 2:
            walls.append(walls[0] if walls else None)
        for i, w in enumerate(walls[:2]):
            if w is None:
                d.wall[i] = dmc_wall(WALL["adiabatic"], 0.0, 0.0)
            else:
                d.wall[i] = dmc_wall(WALL[w.type], float(w.temperature), float(w.specularity))
        h = C.c_void_p()
        dmc_geometry_create(C.byref(d), C.byref(h))
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.dmc_geometry_destroy(self.handle)
        except Exception:
            pass


def job_struct(job, material: Material, keep: list) -> dmc_job:
    """C description of a ``dmc_inputs.Job`` (geometry handle created and kept in ``keep``)."""
    g = Geometry(job.geometry)
    keep.append(g)
    s = dmc_source(SRC[job.source.kind], float(job.source.dT), float(job.source.radius), float(job.source.gradient))
    t = job.tally
    td = dmc_tally_desc()
    td.n_bins, td.n_batches, td.kmax, td.n_hj = int(t.n_bins), int(t.n_batches), int(t.kmax), int(t.n_hj)
    td.first_event = int(bool(getattr(t, "first_event", False)))
    rg = getattr(t, "region", None)
    if rg is not None:
        td.region = 1
        td.region_c[0], td.region_c[1] = float(rg[0]), float(rg[1])
        td.region_radius = float(rg[2])
        td.region_z[0], td.region_z[1] = float(rg[3]), float(rg[4])
    for i in range(3):
        td.grid[i] = int(t.grid[i])
        td.grid_lo[i] = float(t.grid_lo[i])
        td.grid_hi[i] = float(t.grid_hi[i])
    times = np.ascontiguousarray(t.times, np.float64)
    keep.append(times)
    j = dmc_job()
    j.material = material.handle
    j.geometry = g.handle
    j.source = s
    j.tally = td
    j.n_particles = int(job.n_particles)
    j.seed = int(job.seed)
    j.times = _ptr(times, C.c_double) if times.shape[0] else f64p()
    j.n_times = int(times.shape[0])
    j.first_particle = int(getattr(job, "first_particle", 0))
    return j


def run_opts(precision="fp32", form="persistent", stream=None, block=0, chunk=0, refill_min=0, lds_tally=1,
             grid_blocks=0, workspace=None, workspace_bytes=0, nscat_out=None, prio_flights=0,
             nscat_out_len=0) -> dmc_run_opts:
    o = dmc_run_opts()
    dmc_run_opts_default(C.byref(o))
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.form = FORM[form] if isinstance(form, str) else int(form)
    o.stream = stream
    o.block, o.chunk, o.refill_min, o.lds_tally, o.grid_blocks = block, chunk, refill_min, lds_tally, grid_blocks
    o.workspace = workspace
    o.workspace_bytes = workspace_bytes
    o.nscat_out = nscat_out
    o.nscat_out_len = int(nscat_out_len)
    o.prio_flights = int(prio_flights)
    return o


class Result:
    """A launch's results.  ``read(job, quantity)`` returns (mean, stderr) as numpy arrays."""

    def __init__(self, handle: C.c_void_p, jobs: Sequence, keep: list):
        self.handle = handle
        self.jobs = list(jobs)
        self._keep = keep

    def stats(self, job: int = -1) -> dmc_stats:
        s = dmc_stats()
        dmc_result_stats(self.handle, job, C.byref(s))
        return s

    def raw(self, job: int = 0) -> np.ndarray:
        n = C.c_size_t()
        dmc_tally_raw_size(self.handle, job, C.byref(n))
        out = np.zeros(max(n.value, 1))
        dmc_tally_read(self.handle, job, Q_RAW, 0, _ptr(out, C.c_double), f64p(), n.value)
        return out[: n.value]

    def read(self, job: int, quantity: int, time_index: int = 0, n: Optional[int] = None):
        jb = self.jobs[job]
        if n is None:
            if quantity in (Q_T, Q_TLOC, Q_FLUX):
                n = jb.tally.n_bins
            elif quantity == Q_KAPPA:
                n = 1
            elif quantity == Q_HJ:
                n = jb.tally.n_hj
            elif quantity == Q_SNAPSHOT:
                n = int(np.prod(jb.tally.grid))
            elif quantity == Q_SNAPSHOT_SUM:
                n = int(np.prod(jb.tally.grid)) + 1
            elif quantity in (Q_REGION_T, Q_REGION_QZ):
                n = len(jb.tally.times)
            elif quantity in (Q_FIELD_T, Q_FIELD_QZ):
                n = int(jb.tally.grid[0]) * int(jb.tally.grid[2])
            else:
                raise ValueError("give n for this quantity")
        mean = np.zeros(max(n, 1))
        se = np.zeros(max(n, 1))
        dmc_tally_read(self.handle, job, quantity, time_index, _ptr(mean, C.c_double), _ptr(se, C.c_double), n)
        return mean[:n], se[:n]

    def close(self):
        if getattr(self, "handle", None):
            dmc_result_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.dmc_result_destroy(self.handle)
        except Exception:
            pass


def _workspace(workspace):
    """(pointer, bytes) of a caller's device workspace, checked before any library
    call: the library writes there from the device."""
    if workspace is None:
        return None, 0
    if not getattr(workspace, "is_cuda", False) or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    return workspace.data_ptr(), workspace.numel() * workspace.element_size()


def _nscat_buffer(nscat_out, n_total: int):
    """(device pointer, entries) of a per-particle scattering-count tensor: a CUDA
    tensor of a 4-byte integer dtype with at least one entry per particle of the
    launch (the kernels write one uint32 per particle)."""
    if nscat_out is None:
        return None, 0
    if not getattr(nscat_out, "is_cuda", False):
        raise ValueError("nscat_out must be a CUDA tensor")
    if nscat_out.element_size() != 4 or nscat_out.is_floating_point() or not nscat_out.is_contiguous():
        raise ValueError("nscat_out must be a contiguous int32 / uint32 tensor")
    if nscat_out.numel() < n_total:
        raise ValueError(f"nscat_out has {nscat_out.numel()} entries, the launch has {n_total} particles")
    return nscat_out.data_ptr(), int(nscat_out.numel())


def simulate(jobs, material: Optional[Material] = None, precision="fp32", form="persistent", stream=None,
             workspace=None, nscat_out=None, **params) -> Result:
    """Launch ``dmc_inputs.Job`` objects (one launch; they must share a material).

    ``workspace`` may be a CUDA uint8 torch tensor (device memory from torch's
    allocator); ``stream`` a torch.cuda.Stream or raw hipStream_t; ``nscat_out``
    a CUDA uint32/int32 torch tensor with one slot per particle of the launch.
    """
    if not isinstance(jobs, (list, tuple)):
        jobs = [jobs]
    ws_ptr, ws_bytes = _workspace(workspace)
    ns_ptr, ns_len = _nscat_buffer(nscat_out, sum(int(j.n_particles) for j in jobs))
    material = material or Material(jobs[0].material)
    keep: list = [material]
    arr = (dmc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = job_struct(j, material, keep)
    keep.append(arr)
    raw_stream = getattr(stream, "cuda_stream", stream)
    if workspace is not None:
        keep.append(workspace)
    if nscat_out is not None:
        keep.append(nscat_out)
    o = run_opts(precision, form, raw_stream, workspace=ws_ptr, workspace_bytes=ws_bytes, nscat_out=ns_ptr,
                 nscat_out_len=ns_len, **params)
    h = C.c_void_p()
    dmc_simulate_batch(arr, len(jobs), C.byref(o), C.byref(h))
    return Result(h, jobs, keep)


def simulate_one(job, material: Optional[Material] = None, precision="fp32", form="persistent", stream=None,
                 workspace=None, nscat_out=None, **params) -> Result:
    """One ``dmc_inputs.Job`` through ``dmc_simulate`` (the single-simulation entry
    point; whole particle range of the job's seed)."""
    if int(getattr(job, "first_particle", 0)) != 0:
        raise ValueError("dmc_simulate runs whole particle ranges; use simulate() for slices")
    ws_ptr, ws_bytes = _workspace(workspace)
    ns_ptr, ns_len = _nscat_buffer(nscat_out, int(job.n_particles))
    material = material or Material(job.material)
    keep: list = [material]
    j = job_struct(job, material, keep)
    raw_stream = getattr(stream, "cuda_stream", stream)
    if workspace is not None:
        keep.append(workspace)
    if nscat_out is not None:
        keep.append(nscat_out)
    o = run_opts(precision, form, raw_stream, workspace=ws_ptr, workspace_bytes=ws_bytes, nscat_out=ns_ptr,
                 nscat_out_len=ns_len, **params)
    h = C.c_void_p()
    dmc_simulate(j.material, j.geometry, C.byref(j.source), j.n_particles, j.seed, C.byref(j.tally), j.times,
                 j.n_times, C.byref(o), C.byref(h))
    return Result(h, [job], keep)


def noalloc_offsets(jobs, material: Material):
    """Offsets of each job's raw block in the output of simulate_noalloc (n_jobs + 1
    entries; a validation-only call of the entry point)."""
    keep: list = [material]
    arr = (dmc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = job_struct(j, material, keep)
    offs = (C.c_size_t * (len(jobs) + 1))()
    o = run_opts()
    dmc_simulate_batch_noalloc(arr, len(jobs), C.byref(o), None, 0, None, offs)
    return [int(x) for x in offs]


def simulate_noalloc(jobs, raw_out, counters_out=None, material: Optional[Material] = None, precision="fp32",
                     form="persistent", stream=None, nscat_out=None, **params):
    """Enqueue ``jobs`` through dmc_simulate_batch_noalloc: raw tallies into the CUDA
    float64 tensor ``raw_out`` (layout from noalloc_offsets), counters (6 per job,
    dmc_stats order) into the optional CUDA int64 tensor ``counters_out``.
    Asynchronous on ``stream``; returns the offsets."""
    if not isinstance(jobs, (list, tuple)):
        jobs = [jobs]
    material = material or Material(jobs[0].material)
    if not raw_out.is_cuda or raw_out.dtype.itemsize != 8 or not raw_out.is_floating_point() \
            or not raw_out.is_contiguous():
        raise ValueError("raw_out must be a contiguous CUDA float64 tensor")
    if counters_out is not None and (not counters_out.is_cuda or counters_out.element_size() != 8
                                     or counters_out.is_floating_point() or not counters_out.is_contiguous()
                                     or counters_out.numel() < 6 * len(jobs)):
        raise ValueError("counters_out must be a CUDA 64-bit integer tensor of 6 entries per job")
    keep: list = [material]
    arr = (dmc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = job_struct(j, material, keep)
    ns_ptr, ns_len = _nscat_buffer(nscat_out, sum(int(j.n_particles) for j in jobs))
    o = run_opts(precision, form, getattr(stream, "cuda_stream", stream), nscat_out=ns_ptr, nscat_out_len=ns_len,
                 **params)
    offs = (C.c_size_t * (len(jobs) + 1))()
    dmc_simulate_batch_noalloc(arr, len(jobs), C.byref(o), raw_out.data_ptr(), raw_out.numel(),
                               counters_out.data_ptr() if counters_out is not None else None, offs)
    return [int(x) for x in offs]


TUNED_PARAMS = ("block", "chunk", "refill_min", "lds_tally")


def autotune(jobs, material: Optional[Material] = None, precision="fp32", stream=None, sample_flights=0,
             trial_cap=0, use_cache=True):
    """Launch parameters for ``simulate`` chosen by the library's autotuner.

    Returns (params, trials): params is a dict of block / chunk / refill_min /
    lds_tally to pass to ``simulate``; trials lists the timed trials (empty when
    the process-wide cache answered).
    """
    if not isinstance(jobs, (list, tuple)):
        jobs = [jobs]
    material = material or Material(jobs[0].material)
    keep: list = [material]
    arr = (dmc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = job_struct(j, material, keep)
    base = run_opts(precision, "persistent", getattr(stream, "cuda_stream", stream))
    t = dmc_tune_opts()
    t.sample_flights, t.trial_cap, t.use_cache = int(sample_flights), int(trial_cap), int(bool(use_cache))
    buf = (dmc_tune_trial * 64)()
    t.trials = buf
    t.max_trials = 64
    best = dmc_run_opts()
    dmc_autotune(arr, len(jobs), C.byref(base), C.byref(t), C.byref(best))
    trials = [{"block": r.block, "chunk": r.chunk, "refill_min": r.refill_min, "lds_tally": r.lds_tally,
               "pilot": r.pilot, "ms": r.ms, "flights_per_s": r.flights_per_s} for r in buf[:min(t.n_trials, 64)]]
    return {k: int(getattr(best, k)) for k in TUNED_PARAMS}, trials


def plan_truncation(job, material: Optional[Material] = None, precision="fp32", stream=None, n_pilot=0, k_pilot=0,
                    bias_fraction=0.0) -> dict:
    """Truncation K_max for a gradient-source job from a pilot run (see dmc_plan_truncation)."""
    material = material or Material(job.material)
    keep: list = [material]
    j = job_struct(job, material, keep)
    o = run_opts(precision, "persistent", getattr(stream, "cuda_stream", stream))
    t = dmc_trunc_opts()
    t.n_pilot, t.k_pilot, t.bias_fraction = int(n_pilot), int(k_pilot), float(bias_fraction)
    out = dmc_trunc_plan()
    dmc_plan_truncation(C.byref(j), C.byref(o), C.byref(t), C.byref(out))
    return {f: getattr(out, f) for f, _ in dmc_trunc_plan._fields_}


def workspace_bytes(jobs, material: Material, precision="fp32", form="persistent") -> int:
    keep: list = []
    arr = (dmc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = job_struct(j, material, keep)
    o = run_opts(precision, form)
    n = C.c_size_t()
    dmc_workspace_size(arr, len(jobs), C.byref(o), C.byref(n))
    return int(n.value)


def dmc_debug_fp64_math(x, log_out, sin_out, cos_out, n):
    return _call("dmc_debug_fp64_math", x, log_out, sin_out, cos_out, n)


def debug_fp64_math(x):
    """Device FP64 (log x, sin 2 pi x, cos 2 pi x) of the parity mode."""
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[0]
    lg, sn, cs = np.zeros(n), np.zeros(n), np.zeros(n)
    dmc_debug_fp64_math(_ptr(x, C.c_double), _ptr(lg, C.c_double), _ptr(sn, C.c_double), _ptr(cs, C.c_double), n)
    return lg, sn, cs


OP_COSTS = ("fma", "philox_uniform_key", "philox_lane_key", "log", "sin", "cos", "sqrt", "rcp", "f64_add")


def dmc_debug_op_cost(op, iters, blocks, ms, op_count):
    return _call("dmc_debug_op_cost", op, iters, blocks, ms, op_count)


def debug_op_cost(op: str, iters: int, blocks: int = 0):
    """(kernel ms, operations executed) of the instruction-cost probe for ``op``
    (one of OP_COSTS)."""
    ms = C.c_double()
    n = C.c_uint64()
    dmc_debug_op_cost(OP_COSTS.index(op), int(iters), int(blocks), C.byref(ms), C.byref(n))
    return float(ms.value), int(n.value)


def debug_philox(seed: int, pid, k, tag) -> np.ndarray:
    pid = np.ascontiguousarray(pid, np.uint64)
    k = np.ascontiguousarray(k, np.uint32)
    tag = np.ascontiguousarray(tag, np.uint32)
    n = pid.shape[0]
    out = np.zeros((n, 4), np.uint32)
    dmc_debug_philox(int(seed), _ptr(pid, C.c_uint64), _ptr(k, C.c_uint32), _ptr(tag, C.c_uint32),
                     _ptr(out, C.c_uint32), n)
    return out


class Server:
    """Continuous-batching server (dmc_server_*): requests share persistent epoch launches."""

    def __init__(self, material: Material, memory_budget: int, max_active: int = 32, epoch_flights: float = 2e10,
                 drain_flights: int = 0, precision="fp32", stream=None, class_epochs: bool = False, **params):
        o = dmc_server_opts()
        o.memory_budget = int(memory_budget)
        o.max_active = int(max_active)
        o.epoch_flights = int(epoch_flights)
        o.drain_flights = int(drain_flights)
        o.class_epochs = 1 if class_epochs else 0
        o.run = run_opts(precision, "persistent", getattr(stream, "cuda_stream", stream), **params)
        h = C.c_void_p()
        dmc_server_create(material.handle, C.byref(o), C.byref(h))
        self.handle = h
        self.material = material
        self._keep = {}

    def submit(self, job) -> int:
        keep: list = []
        j = job_struct(job, self.material, keep)
        t = C.c_uint64()
        dmc_server_submit(self.handle, C.byref(j), C.byref(t))
        self._keep[t.value] = (job, keep)
        return int(t.value)

    def step(self) -> int:
        n = C.c_int32()
        dmc_server_step(self.handle, C.byref(n))
        return int(n.value)

    def done(self, ticket: int) -> bool:
        d = C.c_int32()
        dmc_server_poll(self.handle, ticket, C.byref(d))
        return bool(d.value)

    def wait(self, ticket: int) -> int:
        """Runs epochs until the ticket's request is complete; returns the epochs run."""
        n = C.c_int32()
        dmc_server_wait(self.handle, ticket, C.byref(n))
        return int(n.value)

    def collect(self, ticket: int) -> Result:
        h = C.c_void_p()
        dmc_server_collect(self.handle, ticket, C.byref(h))
        job, keep = self._keep.pop(ticket)
        return Result(h, [job], keep)

    def load(self):
        q, r = C.c_int32(), C.c_int32()
        dmc_server_load(self.handle, C.byref(q), C.byref(r))
        return int(q.value), int(r.value)

    def totals(self) -> dmc_stats:
        out = dmc_stats()
        dmc_server_totals(self.handle, C.byref(out))
        return out

    def close(self):
        if getattr(self, "handle", None):
            dmc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.dmc_server_destroy(self.handle)
        except Exception:
            pass
