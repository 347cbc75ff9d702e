"""Shared helpers of the GPU tests: the parity cases (small seeded jobs that
the FP64 oracle finishes in seconds, spanning several queue chunks and a
ragged tail) and converters between the oracle's and the library's raw tally
layouts."""
from __future__ import annotations

import numpy as np

import dmc_inputs as di


def small_spot(n=3000, seed=5, grid=16, n_times=8, t_max=5e-11, mat=None):
    job = di.heated_spot(n=n, seed=seed, material=mat or di.silicon_like(), grid=grid, n_times=n_times)
    job.tally.times = tuple(float(t) for t in np.geomspace(1e-12, t_max, n_times))
    return job


def spot_region(n=6000, seed=15):
    """Heated spot with a windowed surface-cylinder tally (a thermoreflectance-like probe)."""
    job = small_spot(n=n, seed=seed, grid=8, n_times=6, t_max=2e-10)
    job.tally.region = (0.0, 0.0, 0.6e-6, 0.0, 0.3e-6)
    job.name = "spot_region"
    return job


def mixed_slab(n=20000, seed=12, mat=None):
    """Hot isothermal wall at z = 0, partly specular adiabatic wall at z = L."""
    mat = mat or di.gray_material()
    g = di.Geometry("slab_z", length=150e-9, walls=[di.Wall("isothermal", 300.5), di.Wall("adiabatic", specularity=0.5)])
    return di.Job(mat, g, di.Source("walls"), di.Tally(n_bins=12), n, seed, "mixed_slab")


def periodic_slab(n=4000, seed=13):
    """Wall-emitted particles in a slab whose other walls re-insert periodically (truncated by kmax)."""
    mat = di.gray_material()
    g = di.Geometry("film_x", length=80e-9, walls=[di.Wall("periodic"), di.Wall("periodic")])
    return di.Job(mat, g, di.Source("gradient", gradient=-1e6), di.Tally(n_bins=10, kmax=12, n_hj=6), n, seed,
                  "periodic_film")


def parity_cases():
    si = di.silicon_like()
    gray = di.gray_material()
    return {
        "gray_slab_C1": di.gray_slab(n=100_000),
        "si_slab_100nm": di.slab_job(si, 100e-9, 20_000, seed=101, n_bins=20),
        "si_slab_1um": di.slab_job(si, 1e-6, 2_000, seed=102, n_bins=20),
        "mixed_slab": mixed_slab(),
        "film_p0.5": di.in_plane_film(60e-9, 0.5, 20_000, seed=103, material=si, kmax=40, n_hj=40, n_bins=8),
        "film_gray_p0": di.in_plane_film(100e-9, 0.0, 20_000, seed=104, material=gray, kmax=10, n_hj=10),
        "film_first_event": di.in_plane_film(60e-9, 0.5, 40_000, seed=107, material=si, kmax=40, n_hj=4,
                                             first_event=True),
        "pore_cell": di.pore_cell(100e-9, 0.3, 20_000, seed=105, material=si, kmax=40, n_hj=40),
        "pore_cell_specular": di.pore_cell(80e-9, 0.2, 10_000, seed=106, material=gray, kmax=20, n_hj=5,
                                           specularity=0.7),
        "pore_field": di.pore_cell(100e-9, 0.3, 20_000, seed=108, material=si, kmax=40, n_hj=8, field=(12, 10)),
        "periodic_film": periodic_slab(),
        "spot": small_spot(),
        "spot_region": spot_region(),
        # Henyey-Greenstein scattering (the generalisation of step IVb): every launch of such a
        # material takes the generic kernel
        "slab_hg": di.slab_job(di.gray_material(scatter_g=-0.4), 150e-9, 20_000, seed=110, n_bins=12),
        "pore_cell_hg": di.pore_cell(100e-9, 0.3, 20_000, seed=109, material=di.silicon_like(scatter_g=0.6),
                                     kmax=40, n_hj=10),
        "spot_hg": small_spot(n=3000, seed=111, mat=di.silicon_like(scatter_g=0.5)),
    }


def lib_sections(job, raw):
    """Split a library raw tally block into the oracle's named sections."""
    t = job.tally
    o = 0
    out = {}
    if t.n_bins > 0:
        n = t.n_batches * 3 * t.n_bins
        out["bins"] = raw[o:o + n].reshape(t.n_batches, 3, t.n_bins)
        o += n
    if job.source.kind == "gradient":
        out["kappa"] = raw[o:o + 2]
        o += 2
        if t.n_hj > 0:
            out["hj"] = raw[o:o + 2 * t.n_hj].reshape(2, t.n_hj)
            o += 2 * t.n_hj
    if len(t.times) > 0:
        nc = int(np.prod(t.grid)) + 1
        nt = len(t.times)
        out["snap"] = raw[o:o + nt * nc].reshape(nt, nc)
        o += nt * nc
        out["snap_abs"] = raw[o:o + nt * nc].reshape(nt, nc)
        o += nt * nc
        if getattr(t, "region", None) is not None:
            out["region"] = raw[o:o + 4 * nt].reshape(nt, 4)
            o += 4 * nt
    elif t.grid[0] > 0:  # steady pore-cell field [batch][TIME, DISPZ][nz][nx]
        nx, nz = int(t.grid[0]), int(t.grid[2])
        n = t.n_batches * 2 * nx * nz
        out["field"] = raw[o:o + n].reshape(t.n_batches, 2, nz, nx)
        o += n
    assert o == raw.shape[0], (o, raw.shape)
    return out


def rel_diff(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = max(float(np.abs(b).max()) if b.size else 0.0, 1e-300)
    return float(np.abs(a - b).max()) / scale if b.size else 0.0


def compare_sections(lib_s, orc_s, rel, vmax=None):
    """Largest relative difference per tally row, and whether all are <= rel.

    Rows: bins per quantity (TIME, PTIME, DISP); kappa and H_j sums and sums of
    squares separately; snapshots.  The DISP row is measured against
    max(|DISP|, 1e-3 vmax max|TIME|): a flux that vanishes by construction (an
    adiabatic wall) leaves only rounding noise, so its scale is the gross
    displacement, not the cancelled sum."""
    worst = {}
    for k, v in lib_s.items():
        ref = orc_s[k]
        if k == "bins":
            for q in range(3):
                d = np.abs(v[:, q, :] - ref[:, q, :]).max()
                scale = np.abs(ref[:, q, :]).max()
                if q == 2 and vmax is not None:
                    scale = max(scale, 1e-3 * vmax * np.abs(ref[:, 0, :]).max())
                worst[f"bins{q}"] = float(d / max(scale, 1e-300))
        elif k == "field":
            for q, name in ((0, "field_time"), (1, "field_dispz")):
                worst[name] = rel_diff(v[:, q], ref[:, q])
        elif k == "region":
            # per window: time and z length in the region, each with its square
            for col, name in enumerate(("region_t", "region_t2", "region_q", "region_q2")):
                worst[name] = rel_diff(v[:, col], ref[:, col])
        elif k in ("kappa", "hj"):
            v2 = np.asarray(v).reshape(2, -1)
            r2 = np.asarray(ref).reshape(2, -1)
            worst[k + "_sum"] = rel_diff(v2[0], r2[0])
            worst[k + "_sq"] = rel_diff(v2[1], r2[1])
        else:
            worst[k] = rel_diff(v, ref)
    return worst, all(w <= rel for w in worst.values())


def vmax_of(job):
    return float(job.material.flat()[3].max())
