"""Pin checks of the FP64 oracle that take the oracle module as an argument.

Each check compares the oracle with something other than itself (a
deterministic solution of the same transport problem, a closed form, a
billiard identity) and raises AssertionError when they disagree.  The tests
call them with the oracle (tests/test_oracle_pins.py) and with copies of it
that carry a deliberately planted mistake (tests/test_oracle_mutants.py), each
of which must fail at least one check.
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy import stats

import dmc_inputs as di
import refsol

THREADS = min(8, os.cpu_count() or 1)


# ------------------------------------------------ frequency-dependent slab ----

def coarse_silicon():
    """Silicon-like material on 40 frequency bins per branch (80 states): free paths
    from 1.9 nm to 0.2 mm, the same dispersion and relaxation-time law as the
    1000-bin material."""
    return di.silicon_like(n_bins=40)


def nongray_reference(orc, L):
    """Bin averages of T and T_loc and the heat flux of the slab integral equation
    (refsol.nongray_slab), Richardson-extrapolated over two meshes (second order)."""
    mat = coarse_silicon()
    om, dom, dos, vg, tau, deg = mat.flat()
    _, Cm, _ = orc.tabulate(mat)
    pb = max(4, int(round(4 * L / 100e-9)))
    T1, P1, q1, _ = refsol.nongray_slab(Cm, vg, tau, L, per_bin=pb)
    T2, P2, q2, q2L = refsol.nongray_slab(Cm, vg, tau, L, per_bin=2 * pb)
    assert abs(q2 - q2L) <= 1e-9 * abs(q2)  # the reference conserves energy
    return (4 * T2 - T1) / 3.0, (4 * P2 - P1) / 3.0, (4 * q2 - q1) / 3.0, abs(q2 - q1)


def check_nongray_slab(orc, L=100e-9, n=200_000, seed=91):
    """Steady frequency-dependent slab between walls at T_eq +- 0.5 K: the
    oracle's bin temperatures, pseudo-temperatures and heat flux agree with the
    deterministic solution of the same linearised problem within 4 standard errors
    (bins: batch means over 16 batches; every bin carries the same flux)."""
    mat = coarse_silicon()
    Tref, Pref, qref, qerr = nongray_reference(orc, L)
    job = di.slab_job(mat, L, n, seed, n_bins=20)
    res, *_ = orc.simulate(job, threads=THREADS)
    for key, ref in (("T", Tref), ("Tloc", Pref)):
        got, se = res[key], res[key + "_se"]
        assert np.all(se < 0.02 * np.abs(ref).max()), (key, se)  # the comparison has teeth
        z = (got - ref) / se
        assert np.all(np.abs(z) < 4.5), (key, L, got, ref, se)
        assert float(np.sum(z ** 2)) < stats.chi2.ppf(0.999, z.size) * 1.5, (key, L, z)
    q, qse = float(res["q"].mean()), float(res["q_se"].mean())
    assert qse < 0.02 * abs(qref)
    assert abs(q - qref) <= 4.0 * qse + 2.0 * qerr, (L, q, qref, qse)


# ----------------------------------------------------------- heated spot ----

# An asymmetric snapshot grid (different cell widths along x and y, off-centre in
# x) so that a transposed cell index or a wrong cell volume shows.
SPOT_GRID = (6, 6, 5)
SPOT_LO = (-1.0e-6, -1.8e-6, 0.0)
SPOT_HI = (2.0e-6, 1.8e-6, 2.5e-6)


def _spot_job(mat, n, seed, times, specularity, grid=SPOT_GRID, lo=SPOT_LO, hi=SPOT_HI, r0=1e-6):
    job = di.heated_spot(n=n, seed=seed, material=mat, grid=4, n_times=len(times), r0=r0, specularity=specularity)
    job.tally.times = tuple(float(t) for t in times)
    job.tally.grid, job.tally.grid_lo, job.tally.grid_hi = tuple(grid), tuple(lo), tuple(hi)
    return job


def _compare_cells(res, ref, what, floor):
    for j in range(ref.shape[0]):
        got = res["snap_T"][j].reshape(ref[j].shape)
        se = res["snap_T_se"][j].reshape(ref[j].shape)
        live = se > 0
        assert np.all(np.abs(got[~live] - ref[j][~live]) <= floor), (what, j)
        z = (got[live] - ref[j][live]) / se[live]
        assert np.all(np.abs(z) < 5.0), (what, j, np.abs(z).max())
        assert float(np.sum(z ** 2)) < stats.chi2.ppf(0.999, z.size) * 1.3, (what, j, float(np.sum(z ** 2)), z.size)


def check_snapshot_ballistic(orc, n=3_000_000, seed=93):
    """Transient estimator of Eq. (3) without scattering (tau = 1 s) and with a
    specular surface: the snapshot temperature of every grid cell at three times
    equals the cell average of the free-streaming solution from the Gaussian
    initial condition (the mean of the mirrored Gaussian over the sphere of radius
    v t), within the per-cell standard errors."""
    v, r0 = 6000.0, 1e-6
    mat = di.gray_material(vg=v, tau=1.0)
    times = (5e-11, 1.5e-10, 3e-10)
    job = _spot_job(mat, n, seed, times, specularity=1.0, r0=r0)
    res, *_ = orc.simulate(job, threads=THREADS)
    ref = np.array([refsol.ballistic_spot_cells(SPOT_GRID, SPOT_LO, SPOT_HI, v, t, r0) for t in times])
    assert float(res["snap_T_se"].max()) < 0.02 * float(ref.max())
    _compare_cells(res, ref, "ballistic", 1e-3 * float(ref.max()))


def check_snapshot_diffusive(orc, n=100_000, seed=94):
    """Transient estimator in the diffusive limit: a gray material with a 1 nm
    free path (v = 1000 m/s, tau = 1 ps) and a Gaussian of radius 30 nm on a
    diffusely reflecting surface; after 340 and 1350 relaxation times the cell
    temperatures near the axis follow Fourier diffusion of the Gaussian with
    alpha = v Lambda / 3 (adiabatic surface by image symmetry)."""
    v, tau, r0 = 1000.0, 1e-12, 30e-9
    alpha = v * v * tau / 3.0
    mat = di.gray_material(vg=v, tau=tau)
    times = (r0 * r0 / (8.0 * alpha), r0 * r0 / (2.0 * alpha))
    grid, lo, hi = (6, 6, 3), (-60e-9, -60e-9, 0.0), (60e-9, 60e-9, 60e-9)
    job = _spot_job(mat, n, seed, times, specularity=0.0, grid=grid, lo=lo, hi=hi, r0=r0)
    res, *_ = orc.simulate(job, threads=THREADS)
    ref = np.array([refsol.diffusive_spot_cells(grid, lo, hi, alpha, t, r0) for t in times])
    # the diffusion solution itself is exact only to O((Lambda / r)^2) and a surface
    # layer of a few free paths: 2 % of the peak is added to each cell's tolerance
    for j in range(len(times)):
        got = res["snap_T"][j].reshape(ref[j].shape)
        se = res["snap_T_se"][j].reshape(ref[j].shape)
        assert float(se.max()) < 0.05 * float(ref[j].max())
        z = (got - ref[j]) / np.hypot(se, 0.02 * ref[j].max() / 2.0)
        assert np.all(np.abs(z) < 4.5), ("diffusive", j, got, ref[j], se)


# ------------------------------------------------------- specular pore ----

def check_specular_pore_chords(orc, porosity=0.3, n=20_000, seed=95):
    """Ballistic walk with specular pore walls: the direction's component along the
    pore axis is conserved, so the x-z projection moves as a two-dimensional
    billiard (the cell's square lattice of discs, a Sinai billiard), whose mean
    free path between collisions is pi A / perimeter (Santalo's formula; A the
    solid area of the cell, perimeter 2 pi r).  The 3-D chord mean is not 4V/S
    here (the axial component is never redistributed), so only the projection is
    checked; 3 % for the heavy-tailed chords of the open channels."""
    job = di.pore_cell(100e-9, porosity, n, seed, material=di.gray_material(), kmax=40, n_hj=0, specularity=1.0)
    prep = orc.prepare(job)
    P, r = job.geometry.length, job.geometry.radius
    m, s3, s2 = orc.pore_chords(prep, 0, job.n_particles, 40)
    assert m > 0.95 * 40 * job.n_particles
    ref2 = math.pi * (P * P - math.pi * r * r) / (2.0 * math.pi * r)
    assert abs((s2 / m) / ref2 - 1.0) < 0.03, (s2 / m, ref2)


# ------------------------------------------------ anisotropic scattering ----

def check_hg_bulk(orc, g=0.6, n=300_000, seed=96):
    """Gray bulk with Henyey-Greenstein scattering: kappa = C v^2 tau / (3 (1 - g))
    within 4 standard errors (a free path keeps g^j of the initial direction after
    j events on average)."""
    mat = di.gray_material(scatter_g=g)
    _, Cm, _ = orc.tabulate(mat)
    om, dom, dos, vg, tau, deg = mat.flat()
    ref = float(np.sum(Cm * vg * vg * tau) / 3.0) / (1.0 - g)
    job = di.pore_cell(200e-9, 0.0, n, seed, material=mat, kmax=60, n_hj=0)
    res, *_ = orc.simulate(job, threads=THREADS)
    assert res["kappa_se"] < 0.02 * ref
    assert abs(res["kappa"] - ref) <= 4 * res["kappa_se"], (res["kappa"], ref, res["kappa_se"])


def _hg_cdf(mu, g):
    return (1.0 - g * g) / (2.0 * g) * ((1.0 + g * g - 2.0 * g * mu) ** -0.5 - 1.0 / (1.0 + g))


def check_hg_sampler(orc, g=0.6, n=40_000, seed=61):
    """Scattering directions for g != 0: unit vectors whose cosine to the incoming
    direction follows the Henyey-Greenstein law (KS against its cumulative
    distribution, mean g, second moment (1 + 2 g^2) / 3), with a uniform azimuth
    (no mean sideways component)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    v = rng.normal(size=(n, 3))
    v[:50] = [0.0, 0.0, 1.0]  # along the frame's axis
    v[50:100] = [0.0, 0.0, -1.0]
    o_in = v / np.linalg.norm(v, axis=1)[:, None]
    o_out = np.array([orc.scatter_direction(g, int(a), int(b), o) for (a, b), o in zip(w, o_in)])
    assert np.allclose(np.linalg.norm(o_out, axis=1), 1.0, atol=1e-12)
    mu = np.sum(o_in * o_out, axis=1)
    assert stats.kstest(mu, lambda m: _hg_cdf(np.asarray(m), g)).pvalue > 1e-3
    assert abs(mu.mean() - g) < 4.0 * mu.std() / math.sqrt(n)
    m2 = np.mean(mu ** 2)
    assert abs(m2 - (1.0 + 2.0 * g * g) / 3.0) < 4.0 * np.std(mu ** 2) / math.sqrt(n)
    side = o_out - mu[:, None] * o_in  # component normal to the incoming direction
    ref = np.cross(o_in, np.array([0.3, -0.5, 0.8]))
    ref /= np.linalg.norm(ref, axis=1)[:, None]
    proj = np.sum(side * ref, axis=1)
    assert abs(proj.mean()) < 4.0 * proj.std() / math.sqrt(n)
