"""Full-size workloads in the launch configuration the benchmark times.

The oracle cannot run these sizes whole, so they are checked three ways:
  * properties that hold at any size: the exact mean number of scattering
    events per particle, the same net displacement in every bin of a slab
    (constant heat flux), antisymmetry of the slab temperature, particle
    conservation and mirror symmetry of the heated spot at every snapshot, and
    the Fuchs-Sondheimer conductivity of in-plane films (exact under the
    truncation, because the flux carried after the first scattering event
    averages to zero in a film);
  * particles sampled from the full-size particle ranges, run as FP64 slices
    and compared with the oracle on the same particle ids (1e-9, >= 99.9 %
    equal scattering counts);
  * pore cells, which have no closed form: the full-size FP32 conductivity
    against the oracle on fewer particles (statistical, with a Bonferroni
    margin over the 40 cells).
"""
import math

import numpy as np
import pytest

import dmc_inputs as di
import oracle
from gpu_cases import compare_sections, lib_sections, rel_diff, vmax_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1206_3316_amd import binding as b  # noqa: E402

import bench  # noqa: E402  (the benchmark's launch configuration)
import refsol  # noqa: E402

THREADS = 16


@pytest.fixture(scope="module")
def si():
    mat = di.silicon_like()
    return mat, b.Material(mat)


def _sums(lm):
    _, s = lm.info()
    return s  # C_tot, G_tau, G_v


def _mean_se(x):
    x = x.double()
    n = x.numel()
    m = float(x.mean())
    v = float(((x - m) ** 2).sum()) / (n - 1)
    return m, math.sqrt(v / n)


def _fp64_slice_matches_oracle(job, first, n, params):
    """Particles first .. first+n-1 of a full-size job: FP64 library vs oracle."""
    sl = di.Job(job.material, job.geometry, job.source, job.tally, n, job.seed, job.name + "_slice", first)
    print(f"slice {job.name} pids {first}..{first + n}", flush=True)
    ns = torch.zeros(n, dtype=torch.int32, device="cuda")
    res = b.simulate([sl], precision="fp64", nscat_out=ns, **params)
    prep = oracle.prepare(sl)
    oraw, ocnt, ons = oracle.run_raw(sl, first, first + n, threads=THREADS, want_nscat=True, prep=prep)
    worst, ok = compare_sections(lib_sections(sl, res.raw(0)), oracle.split_raw(prep, oraw), 1e-9, vmax_of(sl))
    assert ok, (job.name, worst)
    agree = float(np.mean(ns.cpu().numpy() == ons))
    assert agree >= 0.999, (job.name, agree)
    assert res.stats(0).particles == n
    return res


# ------------------------------------------------------- cross-plane films ----

def test_cross_plane_films_full_size(si):
    """12 films x 1e8 particles in one persistent FP32 launch."""
    mat, lm = si
    films = di.cross_plane_films(material=mat)
    params = bench.launch_params(films, lm)
    ntot = sum(j.n_particles for j in films)
    ns = torch.zeros(ntot, dtype=torch.int32, device="cuda")
    print(f"cross-plane films: {ntot} particles, params {params}", flush=True)
    res = b.simulate(films, material=lm, nscat_out=ns, **params)
    C_tot, G_tau, G_v = _sums(lm)
    off = 0
    for j, job in enumerate(films):
        n = job.n_particles
        st = res.stats(j)
        assert st.particles == n and st.capped == 0, job.name
        part = ns[off:off + n]
        off += n
        assert int(part.double().sum()) == st.scatters
        # the mean number of scattering events per particle is 2 L G_tau / G_v exactly
        m, se = _mean_se(part)
        exact = 2.0 * job.geometry.length * G_tau / G_v
        assert abs(m - exact) <= 4.0 * se, (job.name, m, exact, se)
        # every bin carries the same net displacement: constant heat flux
        q, qse = res.read(j, b.Q_FLUX)
        spread = (q.max() - q.min()) / abs(q.mean())
        assert spread <= 1e-4, (job.name, spread)
        assert qse.max() < 0.05 * abs(q.mean())
        # walls at T_eq +- dT: the temperature profile is antisymmetric
        T, Tse = res.read(j, b.Q_T)
        z = (T + T[::-1]) / np.sqrt(Tse ** 2 + Tse[::-1] ** 2)
        assert np.all(np.abs(z) <= 4.5), (job.name, z)


@pytest.mark.parametrize("j", [0, 6, 11])
def test_cross_plane_film_fp64_slices_match_oracle(si, j):
    """The last particles of the 1e8-particle ranges, in FP64, equal the oracle's;
    two adjacent slices add up to their union (how a job shards)."""
    mat, lm = si
    job = di.cross_plane_films(material=mat)[j]
    params = bench.launch_params(di.cross_plane_films(material=mat), lm)
    n = 20_000 if j < 11 else 4_000
    N = job.n_particles
    a = _fp64_slice_matches_oracle(job, N - 2 * n, n, params)
    c = _fp64_slice_matches_oracle(job, N - n, n, params)
    both = di.Job(job.material, job.geometry, job.source, job.tally, 2 * n, job.seed, job.name, N - 2 * n)
    u = b.simulate([both], precision="fp64", **params)
    assert rel_diff(a.raw(0) + c.raw(0), u.raw(0)) <= 1e-12


# ------------------------------------------------------------ heated spot ----

def test_heated_spot_full_size(si):
    """1e9 particles, 64^3 grid x 50 snapshot times, FP32 flight / FP64 tallies."""
    mat, lm = si
    job = di.heated_spot(material=mat, probe=di.TTR_PROBE)
    N = job.n_particles
    params = bench.launch_params([job], lm)
    ns = torch.zeros(N, dtype=torch.int32, device="cuda")
    print(f"heated spot: {N} particles, params {params}", flush=True)
    res = b.simulate([job], material=lm, nscat_out=ns, **params)
    st = res.stats(0)
    assert st.particles == N and st.capped == 0
    C_tot, G_tau, G_v = _sums(lm)
    m, se = _mean_se(ns)
    exact = job.tally.times[-1] * G_tau / C_tot  # E[scatters] = t_final G_tau / C_tot
    assert abs(m - exact) <= 4.0 * se, (m, exact, se)
    g = job.tally.grid[0]
    for ti in range(len(job.tally.times)):
        s, _ = res.read(0, b.Q_SNAPSHOT_SUM, ti)
        assert s.sum() == N, ti  # every particle is in one cell or the overflow slot
        cells = s[:-1].reshape(g, g, g)  # [z][y][x]
        for axis in (1, 2):  # x and y mirror symmetry of the Gaussian spot
            lo = float(np.take(cells, range(g // 2), axis=axis).sum())
            hi = float(np.take(cells, range(g // 2, g), axis=axis).sum())
            assert abs(lo - hi) <= 5.0 * math.sqrt(lo + hi) + 1.0, (ti, axis, lo, hi)
    T, Tse = res.read(0, b.Q_SNAPSHOT, 0)
    assert T.max() > 0.5  # the spot is resolved at 1 ps (dT = 1 K at its centre)
    # the probe cylinder: resolved, and its windowed temperature falls as the heat
    # spreads into the substrate
    Tp, Tpse = res.read(0, b.Q_REGION_T)
    print("probe T", Tp[::7], Tpse[::7], flush=True)
    assert np.all(Tpse[20:] < 0.1 * np.abs(Tp[20:]))
    assert np.all(np.diff(Tp[20:]) < 3.0 * (Tpse[20:][1:] + Tpse[20:][:-1]))


def test_heated_spot_fp64_slice_matches_oracle(si):
    mat, lm = si
    job = di.heated_spot(material=mat)
    params = bench.launch_params([job], lm)
    _fp64_slice_matches_oracle(job, job.n_particles - 2_000, 2_000, params)


# ------------------------------------------------ batched nanostructures ----

def _kappa_fs(mat, d, p):
    Cm = oracle.tabulate(mat)[1]
    om, dom, dos, vg, tau, deg = mat.flat()
    S = refsol.fuchs_sondheimer_S(d / (vg * tau), p)
    return float(np.sum(Cm * vg * vg * tau / 3.0 * S))


def test_batched_nanostructures_full_size(si):
    """64 instances (24 in-plane films, 40 pore cells, 1e6-1e8 particles each) in
    one persistent launch with the autotuned parameters."""
    mat, lm = si
    jobs = di.batched_nanostructures(material=mat)
    params = bench.launch_params(jobs, lm)
    print(f"nanostructures: {sum(j.n_particles for j in jobs)} particles, params {params}", flush=True)
    res = b.simulate(jobs, material=lm, **params)
    z_pore = []
    for i, job in enumerate(jobs):
        st = res.stats(i)
        assert st.particles == job.n_particles and st.capped == 0, job.name
        k, kse = res.read(i, b.Q_KAPPA)
        k, kse = float(k[0]), float(kse[0])
        hj, hse = res.read(i, b.Q_HJ)
        assert abs(hj.sum() - k) <= 1e-9 * abs(k) + 1e-12  # H_j split the conductivity
        if job.geometry.kind == "film_x":
            p = job.geometry.walls[0].specularity
            ref = _kappa_fs(mat, job.geometry.length, p)
            assert kse < 1e-2 * ref, job.name
            assert abs(k - ref) <= max(4.0 * kse, 1e-3 * ref), (job.name, k, ref, kse)
            assert np.all(np.abs(hj[1:]) <= 5.0 * hse[1:]), job.name
        else:
            small = di.Job(job.material, job.geometry, job.source, job.tally, 20_000, job.seed, job.name)
            ores, *_ = oracle.simulate(small, threads=THREADS)
            z_pore.append((k - ores["kappa"]) / math.hypot(kse, ores["kappa_se"]))
    z = np.array(z_pore)
    assert z.shape[0] == 40
    assert np.all(np.abs(z) <= 4.0), z
    assert float(np.sum(z ** 2)) <= 73.4, z  # chi-square, 40 degrees of freedom, 99.9 %


def test_nanostructure_films_first_event_full_size(si):
    """The 24 films of the batch with first-event termination: same
    Fuchs-Sondheimer conductivities, a fraction of the flights."""
    mat, lm = si
    films = [j for j in di.batched_nanostructures(material=mat, first_event_films=True)
             if j.geometry.kind == "film_x"]
    full = [j for j in di.batched_nanostructures(material=mat) if j.geometry.kind == "film_x"]
    assert len(films) == 24
    res = b.simulate(films, material=lm, **bench.launch_params(films, lm))
    ref_run = b.simulate(full, material=lm, **bench.launch_params(full, lm))
    fl_first = sum(res.stats(i).iterations for i in range(24))
    fl_full = sum(ref_run.stats(i).iterations for i in range(24))
    print(f"films: first-event {fl_first:.3e} flights in {res.stats(0).kernel_ms:.1f} ms, "
          f"K_max = 40 {fl_full:.3e} flights in {ref_run.stats(0).kernel_ms:.1f} ms", flush=True)
    assert fl_first < 0.5 * fl_full
    for i, job in enumerate(films):
        st = res.stats(i)
        assert st.particles == job.n_particles and st.capped == 0 and st.scatters <= job.n_particles
        k, kse = res.read(i, b.Q_KAPPA)
        ref = _kappa_fs(mat, job.geometry.length, job.geometry.walls[0].specularity)
        assert kse[0] < 1e-2 * ref, job.name
        assert abs(k[0] - ref) <= max(4.0 * kse[0], 1e-3 * ref), (job.name, k[0], ref, kse[0])


@pytest.mark.parametrize("i", [0, 23, 24, 63])
def test_batched_nanostructure_fp64_slices_match_oracle(si, i):
    mat, lm = si
    jobs = di.batched_nanostructures(material=mat)
    params = bench.launch_params(jobs, lm)
    job = jobs[i]
    _fp64_slice_matches_oracle(job, job.n_particles - 5_000, 5_000, params)
