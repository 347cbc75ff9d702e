"""FP64 CPU oracle of the linearized deviational phonon Monte Carlo method.

TEST INFRASTRUCTURE ONLY: the plain, slow reference that the GPU library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product path never does.
It shares no code with ``paper_1206_3316_amd`` (only the seeded problem
descriptions of ``dmc_inputs`` are common to both).

Layers:
  * ``dmc_oracle.c``   -- Philox, heat-capacity tabulation, alias tables and
    steps I-VI with the estimators, all FP64 (see that file's header);
  * this module        -- ctypes marshalling, the source normalisations of the
    source-term paragraph (N = total deviational energy / E_eff, steady power
    E_eff / T) and the conversion of raw sums into temperatures, heat fluxes,
    conductivities and standard errors.

The pore-cell geometry has no printed value; it is pinned by brute-force ray
marching of the boundary search, the area law of the emitted positions and
Cauchy's mean chord formula for a ballistic walk (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

import dmc_inputs as di

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmc_oracle.c")
_LIB = os.path.join(_HERE, "_dmc_oracle.so")

GEOM = {"slab_z": 0, "film_x": 1, "pore_cell_xz": 2, "halfspace_z": 3}
WALL = {"isothermal": 0, "adiabatic": 1, "periodic": 2}
SRC = {"walls": 0, "gaussian": 1, "gradient": 2}
TAG_STEP, TAG_EMIT_A, TAG_EMIT_B = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [
        ("K", C.c_int32),
        ("v", C.POINTER(C.c_double)), ("tau", C.POINTER(C.c_double)),
        ("gain_bits", C.c_int32), ("gain_thresh", C.POINTER(C.c_uint32)), ("gain_alias", C.POINTER(C.c_uint32)),
        ("init_bits", C.c_int32), ("init_thresh", C.POINTER(C.c_uint32)), ("init_alias", C.POINTER(C.c_uint32)),
        ("flux_bits", C.c_int32), ("flux_thresh", C.POINTER(C.c_uint32)), ("flux_alias", C.POINTER(C.c_uint32)),
        ("n_src", C.c_int32), ("src_bits", C.c_int32), ("src_thresh", C.POINTER(C.c_uint32)),
        ("src_alias", C.POINTER(C.c_uint32)), ("src_wall", C.POINTER(C.c_int32)),
        ("geom", C.c_int32), ("length", C.c_double), ("radius", C.c_double),
        ("wall_type", C.c_int32 * 2), ("wall_T", C.c_double * 2), ("wall_spec", C.c_uint64 * 2),
        ("src_kind", C.c_int32), ("T_eq", C.c_double), ("dT", C.c_double), ("r0", C.c_double), ("G", C.c_double),
        ("n_bins", C.c_int32), ("n_batches", C.c_int32), ("kmax", C.c_int32), ("n_hj", C.c_int32),
        ("n_times", C.c_int32), ("times", C.POINTER(C.c_double)),
        ("grid", C.c_int32 * 3), ("grid_lo", C.c_double * 3), ("grid_hi", C.c_double * 3),
        ("seed", C.c_uint64),
        ("first_event", C.c_int32),
        ("region_kind", C.c_int32), ("region_c", C.c_double * 2), ("region_r", C.c_double),
        ("region_z", C.c_double * 2),
        ("field_n", C.c_int32 * 2), ("field_lo", C.c_double * 2), ("field_hi", C.c_double * 2),
        ("scatter_g", C.c_double),
    ]


class Counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in
                ("particles", "scatters", "boundary", "iterations", "absorbed", "capped", "periodic")]


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = C.CDLL(_LIB)
            u32p, f64p = C.POINTER(C.c_uint32), C.POINTER(C.c_double)
            L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
            L.oracle_rng_block.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, u32p]
            L.oracle_tabulate.argtypes = [C.c_int32] + [f64p] * 6 + [C.c_double, f64p, f64p, f64p]
            L.oracle_tabulate.restype = C.c_int
            L.oracle_alias_bits.argtypes = [C.c_int32]
            L.oracle_alias_bits.restype = C.c_int32
            L.oracle_alias.argtypes = [C.c_int32, f64p, C.POINTER(C.c_uint64), u32p, u32p]
            L.oracle_alias.restype = C.c_int32
            L.oracle_tally_size.argtypes = [C.POINTER(Problem)]
            L.oracle_tally_size.restype = C.c_size_t
            L.oracle_run.argtypes = [C.POINTER(Problem), C.c_uint64, C.c_uint64, f64p, C.POINTER(Counters), u32p,
                                     C.POINTER(C.c_uint64)]
            L.oracle_run.restype = C.c_int
            L.oracle_log.argtypes = [C.c_double]
            L.oracle_log.restype = C.c_double
            L.oracle_sincos2pi.argtypes = [C.c_double, f64p, f64p]
            L.oracle_boundary_search.argtypes = [C.POINTER(Problem), f64p, f64p, C.c_double, C.c_int32,
                                                 C.POINTER(C.c_int32)]
            L.oracle_boundary_search.restype = C.c_double
            L.oracle_emit.argtypes = [C.POINTER(Problem), C.c_uint64, f64p, f64p, u32p, f64p]
            L.oracle_pore_chords.argtypes = [C.POINTER(Problem), C.c_uint64, C.c_uint64, C.c_uint32, f64p, f64p]
            L.oracle_pore_chords.restype = C.c_uint64
            L.oracle_scatter_direction.argtypes = [C.c_double, C.c_uint32, C.c_uint32, f64p, f64p]
            _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# --------------------------------------------------------------------------
# Low-level pieces (exposed for the pin tests)
# --------------------------------------------------------------------------


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def rng_block(seed: int, pid: int, k: int, tag: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_rng_block(seed, pid, k, tag, _p(out, C.c_uint32))
    return out


def log(x: float) -> float:
    """The reference's logarithm (IEEE basic operations only)."""
    return lib().oracle_log(float(x))


def sincos2pi(u: float):
    """The reference's (sin, cos) of 2 pi u (IEEE basic operations only)."""
    s, c = C.c_double(), C.c_double()
    lib().oracle_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def tabulate(material: di.Material):
    """Per-state (dedT, C) and the sums (C_tot, G_tau = sum C/tau, G_v = sum C v)."""
    om, dom, dos, vg, tau, deg = material.flat()
    K = om.shape[0]
    dedT = np.zeros(K)
    Cm = np.zeros(K)
    sums = np.zeros(3)
    rc = lib().oracle_tabulate(K, _p(om, C.c_double), _p(dom, C.c_double), _p(dos, C.c_double),
                               _p(vg, C.c_double), _p(tau, C.c_double), _p(deg, C.c_double), material.T_eq,
                               _p(dedT, C.c_double), _p(Cm, C.c_double), _p(sums, C.c_double))
    if rc != 0:
        raise ValueError("oracle: invalid material")
    return dedT, Cm, sums


def alias(weights) -> Dict[str, np.ndarray]:
    """Alias table of the weights: bits b, integer masses q (sum 2^32), thresh, alias."""
    w = np.ascontiguousarray(weights, dtype=np.float64)
    K = w.shape[0]
    b = lib().oracle_alias_bits(K)
    n = 1 << b
    q = np.zeros(n, np.uint64)
    th = np.zeros(n, np.uint32)
    al = np.zeros(n, np.uint32)
    rb = lib().oracle_alias(K, _p(w, C.c_double), _p(q, C.c_uint64), _p(th, C.c_uint32), _p(al, C.c_uint32))
    if rb < 0:
        raise ValueError("oracle: invalid alias weights")
    return {"bits": rb, "q": q, "thresh": th, "alias": al}


def alias_draw(table, words: np.ndarray) -> np.ndarray:
    """Vectorised lookup of the alias table for uint32 words (same rule as the C side)."""
    w = np.asarray(words, dtype=np.uint64)
    b = table["bits"]
    idx = (w >> np.uint64(32 - b)).astype(np.int64)
    low = w & np.uint64((1 << (32 - b)) - 1)
    keep = low < table["thresh"][idx].astype(np.uint64)
    return np.where(keep, idx, table["alias"][idx].astype(np.int64))


# --------------------------------------------------------------------------
# Problem preparation: tabulation, alias tables, source normalisation
# --------------------------------------------------------------------------


@dataclass
class Prepared:
    job: di.Job
    struct: Problem
    keep: list  # arrays referenced by the struct
    C_tot: float
    G_tau: float
    G_v: float
    power: float  # steady: total source power per unit area / length; transient: total energy
    steady: bool
    avg_volume: float  # mu(R) of the conductivity average
    tally_size: int


def prepare(job: di.Job) -> Prepared:
    mat, g, src, tl = job.material, job.geometry, job.source, job.tally
    om, dom, dos, vg, tau, deg = mat.flat()
    dedT, Cm, sums = tabulate(mat)
    C_tot, G_tau, G_v = (float(x) for x in sums)
    gain = alias(Cm / tau)
    init = alias(Cm)
    flux = alias(Cm * vg)
    keep = [vg, tau, gain, init, flux]
    P = Problem()
    P.K = om.shape[0]
    P.v, P.tau = _p(vg, C.c_double), _p(tau, C.c_double)
    for name, t in (("gain", gain), ("init", init), ("flux", flux)):
        setattr(P, name + "_bits", t["bits"])
        setattr(P, name + "_thresh", _p(t["thresh"], C.c_uint32))
        setattr(P, name + "_alias", _p(t["alias"], C.c_uint32))
    if g.kind not in GEOM:
        raise ValueError(f"unknown geometry {g.kind}")
    P.geom = GEOM[g.kind]
    P.length, P.radius = float(g.length), float(g.radius)
    walls = list(g.walls) + [di.Wall("adiabatic")] * (2 - len(g.walls))
    for i in range(2):
        P.wall_type[i] = WALL[walls[i].type]
        P.wall_T[i] = float(walls[i].temperature)
        P.wall_spec[i] = min(int(round(walls[i].specularity * 2.0 ** 32)), 1 << 32)
    P.src_kind = SRC[src.kind]
    P.T_eq = float(mat.T_eq)
    P.dT, P.r0, P.G = float(src.dT), float(src.radius), float(src.gradient)

    steady = len(tl.times) == 0
    avg_volume = 1.0
    if src.kind == "walls":
        # isothermal wall at T_b emits V_g cos(theta) C_{w,p} |T_b - T_eq| into its half
        # space: the hemisphere integral of cos(theta)/(4 pi) is 1/4
        if g.kind not in ("slab_z", "film_x"):
            raise ValueError("wall sources need a slab or film geometry")
        powers, wall_ids = [], []
        for i, w in enumerate(walls):
            if w.type == "isothermal" and w.temperature != mat.T_eq:
                powers.append(abs(w.temperature - mat.T_eq) * G_v / 4.0)
                wall_ids.append(i)
        if not powers:
            raise ValueError("no emitting wall")
        power = float(sum(powers))
        srct = alias(np.array(powers))
        wall_arr = np.array(wall_ids, np.int32)
        keep += [srct, wall_arr]
        P.n_src = len(powers)
        P.src_bits, P.src_thresh, P.src_alias = srct["bits"], _p(srct["thresh"], C.c_uint32), _p(srct["alias"], C.c_uint32)
        P.src_wall = _p(wall_arr, C.c_int32)
        avg_volume = g.length
    elif src.kind == "gradient":
        # -D/(4 pi) V_g cos(theta) de/dT dT/dz: the sphere integral of |cos(theta)|/(4 pi) is 1/2
        if g.kind == "film_x":
            vol = g.length
            avg_volume = g.length
        elif g.kind == "pore_cell_xz":
            vol = g.length ** 2 - math.pi * g.radius ** 2
            avg_volume = g.length ** 2
        else:
            raise ValueError("gradient sources need a film or pore-cell geometry")
        if src.gradient == 0.0:
            raise ValueError("zero gradient")
        power = vol * abs(src.gradient) * G_v / 2.0
        P.n_src = 1
    else:  # gaussian initial condition on the half space: C_tot dT pi^{3/2} r0^3 / 2
        if g.kind != "halfspace_z" or steady:
            raise ValueError("the gaussian initial condition needs a half space and snapshot times")
        power = C_tot * abs(src.dT) * math.pi ** 1.5 * src.radius ** 3 / 2.0
        P.n_src = 1
    P.n_bins, P.n_batches, P.kmax, P.n_hj = int(tl.n_bins), int(tl.n_batches), int(tl.kmax), int(tl.n_hj)
    P.first_event = int(bool(getattr(tl, "first_event", False)))
    if P.first_event and (job.geometry.kind != "film_x" or job.source.kind != "gradient"):
        raise ValueError("first-event termination applies to in-plane films under the gradient source")
    P.scatter_g = float(getattr(mat, "scatter_g", 0.0))
    if not -1.0 < P.scatter_g < 1.0:
        raise ValueError("the mean scattering cosine g must lie in (-1, 1)")
    if P.first_event and P.scatter_g != 0.0:
        raise ValueError("first-event termination needs isotropic scattering (the flux after a scattering "
                         "event averages to zero only then)")
    if tl.kmax >= 0 and tl.n_hj > tl.kmax:
        raise ValueError("n_hj must not exceed kmax")
    times = np.ascontiguousarray(tl.times, dtype=np.float64)
    keep.append(times)
    P.n_times = times.shape[0]
    P.times = _p(times, C.c_double) if times.shape[0] else C.POINTER(C.c_double)()
    for d in range(3):
        P.grid[d] = int(tl.grid[d]) if not steady else 0
        P.grid_lo[d], P.grid_hi[d] = float(tl.grid_lo[d]), float(tl.grid_hi[d])
    if steady and tl.grid[0] > 0:
        # steady pore cell: an x-z field over the unit cell (y is the cell's axis of invariance)
        if g.kind != "pore_cell_xz" or tl.grid[1] != 1 or tl.grid[2] < 1:
            raise ValueError("a steady field needs a pore cell and grid (nx, 1, nz)")
        if (tl.grid_lo[0], tl.grid_lo[2], tl.grid_hi[0], tl.grid_hi[2]) != (0.0, 0.0, g.length, g.length):
            raise ValueError("a steady field covers the unit cell [0, P) x [0, P)")
        P.field_n[0], P.field_n[1] = int(tl.grid[0]), int(tl.grid[2])
        P.field_lo[0], P.field_lo[1] = 0.0, 0.0
        P.field_hi[0], P.field_hi[1] = float(g.length), float(g.length)
    P.seed = int(job.seed)
    rg = getattr(tl, "region", None)
    if rg is not None:
        if steady:
            raise ValueError("the windowed region tally needs snapshot times")
        P.region_kind = 1
        P.region_c[0], P.region_c[1] = float(rg[0]), float(rg[1])
        P.region_r = float(rg[2])
        P.region_z[0], P.region_z[1] = float(rg[3]), float(rg[4])
    size = int(lib().oracle_tally_size(C.byref(P)))
    return Prepared(job, P, keep, C_tot, G_tau, G_v, power, steady, avg_volume, size)


def boundary_search(prep: "Prepared", x, o, v: float = 1.0, last: int = -1):
    """Step III for one state: (hit time, surface index); surface -1 and an
    infinite time when the ray meets no surface."""
    xa = np.ascontiguousarray(x, dtype=np.float64)
    oa = np.ascontiguousarray(o, dtype=np.float64)
    surf = C.c_int32(0)
    t = lib().oracle_boundary_search(C.byref(prep.struct), _p(xa, C.c_double), _p(oa, C.c_double), float(v),
                                     int(last), C.byref(surf))
    return float(t), int(surf.value)


def emit_state(prep: "Prepared", pid: int):
    """Step I for one particle id: (position, direction, state, sign)."""
    x = np.zeros(3)
    o = np.zeros(3)
    m = C.c_uint32(0)
    s = C.c_double(0.0)
    lib().oracle_emit(C.byref(prep.struct), int(pid), _p(x, C.c_double), _p(o, C.c_double), C.byref(m), C.byref(s))
    return x, o, int(m.value), float(s.value)


def scatter_direction(g: float, w2: int, w3: int, o_in) -> np.ndarray:
    """Step IVb's new direction for incoming direction o_in and words w2, w3."""
    oi = np.ascontiguousarray(o_in, dtype=np.float64)
    out = np.zeros(3)
    lib().oracle_scatter_direction(float(g), int(w2), int(w3), _p(oi, C.c_double), _p(out, C.c_double))
    return out


def pore_chords(prep: "Prepared", pid_begin: int, pid_end: int, n_chords: int):
    """Ballistic walk in a pore cell (see oracle_pore_chords): (number of chords
    between consecutive pore hits, sum of their lengths, sum of their x-z
    projections)."""
    s3 = C.c_double(0.0)
    s2 = C.c_double(0.0)
    n = lib().oracle_pore_chords(C.byref(prep.struct), int(pid_begin), int(pid_end), int(n_chords), C.byref(s3),
                                 C.byref(s2))
    return int(n), float(s3.value), float(s2.value)


# --------------------------------------------------------------------------
# Running and finalising
# --------------------------------------------------------------------------


def run_raw(job: di.Job, pid_begin: int = 0, pid_end: Optional[int] = None, threads: int = 1,
            want_nscat: bool = False, prep: Optional[Prepared] = None, hist: Optional[np.ndarray] = None):
    """Run particles [pid_begin, pid_end) and return (raw tally, counters dict, nscat or None).

    Threads take contiguous pid ranges with private tallies summed in range order.
    ``hist`` (uint64, one slot per state) receives the post-scattering state counts.
    """
    prep = prep or prepare(job)
    pid_end = job.n_particles if pid_end is None else pid_end
    n = pid_end - pid_begin
    threads = max(1, min(threads, n)) if n > 0 else 1
    cuts = [pid_begin + (n * i) // threads for i in range(threads + 1)]
    tallies = [np.zeros(prep.tally_size) for _ in range(threads)]
    hists = [np.zeros(prep.struct.K, np.uint64) for _ in range(threads)] if hist is not None else None
    cnts = [Counters() for _ in range(threads)]
    nscat = np.zeros(max(n, 1), np.uint32) if want_nscat else None

    def work(i):
        a, b = cuts[i], cuts[i + 1]
        out = _p(nscat[a - pid_begin:], C.c_uint32) if want_nscat else C.POINTER(C.c_uint32)()
        hp = _p(hists[i], C.c_uint64) if hists is not None else C.POINTER(C.c_uint64)()
        rc = lib().oracle_run(C.byref(prep.struct), a, b, _p(tallies[i], C.c_double), C.byref(cnts[i]), out, hp)
        if rc != 0:
            raise RuntimeError("oracle_run failed")

    if threads == 1:
        work(0)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(threads)))
    raw = np.zeros(prep.tally_size)
    for t in tallies:
        raw += t
    if hist is not None:
        for h in hists:
            hist += h
    counters = {f: sum(getattr(c, f) for c in cnts) for f, _ in Counters._fields_}
    return raw, counters, (nscat[:n] if want_nscat else None)


def split_raw(prep: Prepared, raw: np.ndarray) -> Dict[str, np.ndarray]:
    tl = prep.job.tally
    B, nb = tl.n_batches, tl.n_bins
    o = 0
    out = {}
    out["bins"] = raw[o:o + B * 3 * nb].reshape(B, 3, nb); o += B * 3 * nb
    out["kappa"] = raw[o:o + 2]; o += 2
    out["hj"] = raw[o:o + 2 * tl.n_hj].reshape(2, tl.n_hj); o += 2 * tl.n_hj
    nt = len(tl.times) if not prep.steady else 0
    ncell = int(np.prod(tl.grid)) if nt else 0
    out["snap"] = raw[o:o + nt * (ncell + 1)].reshape(nt, ncell + 1); o += nt * (ncell + 1)
    out["snap_abs"] = raw[o:o + nt * (ncell + 1)].reshape(nt, ncell + 1); o += nt * (ncell + 1)
    if getattr(tl, "region", None) is not None and nt:
        out["region"] = raw[o:o + 4 * nt].reshape(nt, 4); o += 4 * nt
    if prep.steady and tl.grid[0] > 0:
        nx, nz = int(tl.grid[0]), int(tl.grid[2])
        out["field"] = raw[o:o + B * 2 * nx * nz].reshape(B, 2, nz, nx); o += B * 2 * nx * nz
    return out


def batch_counts(N: int, B: int) -> np.ndarray:
    """Particles per batch when batch = pid mod B."""
    return np.array([(N - b + B - 1) // B if N > b else 0 for b in range(B)], dtype=np.float64)


def finalize(prep: Prepared, raw: np.ndarray, N: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Physical results from the raw sums (FP64).

    Steady (Eq. (4)): E_dot = power / N; bin energy density E_dot sum(s t_k) / dz,
    dT = that / C_tot, pseudo-temperature with G_tau, heat flux E_dot sum(s dz_k) / dz.
    Conductivity: mean flux E_dot sum(s L_i) / mu(R), kappa = -q / (dT/dz).
    Transient (Eq. (3)): E_eff = E / N; dT(cell) = E_eff sum(s) / (V_cell C_tot).
    Standard errors: batch means for bins, per-particle moments otherwise.
    """
    job = prep.job
    tl = job.tally
    N = job.n_particles if N is None else N
    parts = split_raw(prep, raw)
    res: Dict[str, np.ndarray] = {}
    if tl.n_bins > 0:
        dz = job.geometry.length / tl.n_bins
        nbat = batch_counts(N, tl.n_batches)
        scale = np.array([1.0 / prep.C_tot, 1.0 / prep.G_tau, 1.0]) * prep.power / dz
        tot = parts["bins"].sum(axis=0)  # (3, nb)
        mean = tot * scale[:, None] / N
        good = nbat > 0
        per = parts["bins"][good] * scale[None, :, None] / nbat[good][:, None, None]
        nb_good = int(good.sum())
        se = per.std(axis=0, ddof=1) / math.sqrt(nb_good) if nb_good > 1 else np.full_like(mean, np.nan)
        for i, name in enumerate(("T", "Tloc", "q")):
            res[name] = mean[i]
            res[name + "_se"] = se[i]
    if job.source.kind == "gradient":
        s1, s2 = parts["kappa"]
        G = job.source.gradient
        f = prep.power / (prep.avg_volume * G)  # kappa = -f * mean(L)
        m = s1 / N
        var = max(s2 / N - m * m, 0.0)
        res["kappa"] = np.array(-f * m)
        res["kappa_se"] = np.array(abs(f) * math.sqrt(var / max(N - 1, 1)))
        if tl.n_hj > 0:
            h1, h2 = parts["hj"]
            hm = h1 / N
            hv = np.maximum(h2 / N - hm * hm, 0.0)
            res["hj"] = -f * hm
            res["hj_se"] = abs(f) * np.sqrt(hv / max(N - 1, 1))
    if "field" in parts:
        # steady field (Eq. (4) per cell, per unit length along y): T = E_dot sum(s t_c) / (A_c C_tot),
        # q_z = E_dot sum(s v Omega_z t_c) / A_c with A_c the full cell area; batch means for the SE
        nz, nx = parts["field"].shape[2:]
        area = (job.geometry.length / nx) * (job.geometry.length / nz)
        nbat = batch_counts(N, tl.n_batches)
        good = nbat > 0
        for name, q, den in (("field_T", 0, area * prep.C_tot), ("field_q", 1, area)):
            F = parts["field"][:, q]  # (B, nz, nx)
            res[name] = prep.power * F.sum(axis=0) / (N * den)
            per = prep.power * F[good] / (nbat[good][:, None, None] * den)
            ng = int(good.sum())
            res[name + "_se"] = per.std(axis=0, ddof=1) / math.sqrt(ng) if ng > 1 else np.full((nz, nx), np.nan)
    if not prep.steady:
        g = np.array(tl.grid, dtype=np.float64)
        vcell = float(np.prod((np.array(tl.grid_hi) - np.array(tl.grid_lo)) / g))
        e_eff = prep.power / N
        S, A = parts["snap"], parts["snap_abs"]
        res["snap_T"] = e_eff * S[:, :-1] / (vcell * prep.C_tot)
        var = np.maximum(A / N - (S / N) ** 2, 0.0)
        res["snap_T_se"] = e_eff * N * np.sqrt(var[:, :-1] / N) / (vcell * prep.C_tot)
        res["snap_overflow"] = S[:, -1]
        res["snap_sum"] = S.sum(axis=1)
        if "region" in parts:
            # time average over window [t_{j-1}, t_j): E_eff sum_i s_i (time in R) / (T_w mu(R) C_tot);
            # heat flux E_eff sum_i s_i (z displacement in R) / (T_w mu(R)); per-particle moments for SE
            rg = tl.region
            mu = math.pi * rg[2] ** 2 * (rg[4] - rg[3])
            edges = np.concatenate([[0.0], np.asarray(tl.times, dtype=np.float64)])
            tw = np.diff(edges)
            R = parts["region"]
            for key, col, den in (("region_T", 0, mu * prep.C_tot), ("region_q", 2, mu)):
                m = R[:, col] / N
                v = np.maximum(R[:, col + 1] / N - m * m, 0.0) * N / max(N - 1, 1)
                res[key] = e_eff * R[:, col] / (tw * den)
                res[key + "_se"] = e_eff * np.sqrt(N * v) / (tw * den)
    return res


def simulate(job: di.Job, threads: int = 1, want_nscat: bool = False, n: Optional[int] = None):
    """Run the whole job (or its first ``n`` particles) and finalise.  Returns (results, raw, counters, nscat)."""
    prep = prepare(job)
    N = job.n_particles if n is None else n
    raw, cnt, ns = run_raw(job, 0, N, threads, want_nscat, prep)
    return finalize(prep, raw, N), raw, cnt, ns
