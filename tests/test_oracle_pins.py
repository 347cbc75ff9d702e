"""Pins of the FP64 CPU oracle against things other than itself.

Each test names what it checks the oracle against: an independent black-box
implementation (rocRAND's Philox), exact integer identities, a finite
difference, closed-form limits, deterministic integral-equation solutions of
the same transport problem (tests/refsol.py), exact invariants of the method,
and chi-square agreement of sampled states with the normalised gain
distribution of Eq. (2).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import dmc_inputs as di
import oracle
import refsol

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = min(8, os.cpu_count() or 1)


# ---------------------------------------------------------------- Philox ----

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_ref.cpp")])
    return exe


def test_philox_matches_rocrand_black_box(rocrand_ref):
    """Raw Philox4x32-10 blocks equal rocRAND's engine positioned at the same counter/key."""
    rng = np.random.Generator(np.random.PCG64(123))
    n = 20000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 29) - 1  # rocRAND's offset argument counts 32-bit words
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    edges = [([0, 0, 0, 0], [0, 0]), ([2 ** 32 - 1, 0, 2 ** 32 - 1, 2 ** 32 - 1], [2 ** 32 - 1, 2 ** 32 - 1]),
             ([1, 0, 0, 0], [0, 0]), ([0, 0, 0, 1], [0, 0]), ([0, 0, 1, 0], [1, 0])]
    ctr = np.vstack([ctr, np.array([e[0] for e in edges], np.uint64)])
    key = np.vstack([key, np.array([e[1] for e in edges], np.uint64)])
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    got = np.array([oracle.philox(c, k) for c, k in zip(ctr, key)], dtype=np.uint64)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_rng_block_counter_layout():
    """(seed, pid, k, tag) map onto key = seed words and counter = (pid lo, pid hi, k, tag)."""
    seed, pid, k, tag = 0x0123456789ABCDEF, 0x00000002FFFFFFFE, 77, 2
    a = oracle.rng_block(seed, pid, k, tag)
    b = oracle.philox([pid & 0xFFFFFFFF, pid >> 32, k, tag], [seed & 0xFFFFFFFF, seed >> 32])
    assert np.array_equal(a, b)


def test_uniform_words_statistics():
    """Philox words behave as independent uniforms (KS on the open-interval map)."""
    w = np.array([oracle.rng_block(9, pid, 0, 0) for pid in range(5000)], dtype=np.float64)
    u = (w + 0.5) / 2.0 ** 32
    for col in range(4):
        assert stats.kstest(u[:, col], "uniform").pvalue > 1e-3


# ------------------------------------------------- elementary functions ----

def _ulps(a, b):
    return abs(a - b) / np.spacing(abs(b))


def test_reference_log_within_one_ulp_of_libm():
    """The reference logarithm (atanh series on IEEE basic operations) agrees with the C
    library to about an ulp over the whole range of R = (w + 1/2) 2^-32."""
    rng = np.random.Generator(np.random.PCG64(8))
    w = np.concatenate([rng.integers(0, 2 ** 32, 20000), [0, 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2, 3037000499]])
    worst = 0.0
    for wi in w:
        u = (float(wi) + 0.5) / 2.0 ** 32
        worst = max(worst, _ulps(oracle.log(u), math.log(u)))
    assert worst <= 2.0, worst
    for x in (1e-300, 0.5, 1.0, 2.0, math.e, 1e300):
        assert _ulps(oracle.log(x), math.log(x)) <= 2.0 or abs(math.log(x)) < 1e-300


def test_reference_sincos_2pi_accuracy_and_symmetries():
    """sin/cos of 2 pi u within 2e-16 of the C library, exact at quarter turns."""
    rng = np.random.Generator(np.random.PCG64(9))
    us = np.concatenate([rng.random(20000), [0.0, 0.125, 0.25, 0.5, 0.75, 0.999999999, 1e-12, 0.3749999999]])
    for u in us:
        s, c = oracle.sincos2pi(u)
        assert abs(s - math.sin(2 * math.pi * u)) <= 2e-16 + 1e-15 * abs(u)
        assert abs(c - math.cos(2 * math.pi * u)) <= 2e-16 + 1e-15 * abs(u)
    assert oracle.sincos2pi(0.25) == (1.0, 0.0) or oracle.sincos2pi(0.25)[0] == 1.0
    assert oracle.sincos2pi(0.5)[1] == -1.0 and oracle.sincos2pi(0.0) == (0.0, 1.0)


# ---------------------------------------------------------- Tabulation ----

HBAR, KB = 1.054571817e-34, 1.380649e-23


def _bose_energy(omega, T):
    return HBAR * omega / np.expm1(HBAR * omega / (KB * T))


def test_dedT_matches_finite_difference():
    """de^eq/dT equals a central difference of the Bose-Einstein mode energy."""
    om = np.array([1e11, 3e12, 1e13, 5e13, 7.6e13])
    for T in (4.0, 77.0, 300.0, 1000.0):
        mat = di.Material([di.Branch(om, np.ones(5), np.ones(5), np.full(5, 5e3), np.full(5, 1e-11), 1.0)], T_eq=T)
        dedT, Cm, sums = oracle.tabulate(mat)
        h = T * 1e-5
        fd = (_bose_energy(om, T + h) - _bose_energy(om, T - h)) / (2 * h)
        ok = fd > 1e-300
        assert np.allclose(dedT[ok], fd[ok], rtol=1e-7)
        assert np.array_equal(Cm, dedT)  # D = domega = g = 1


def test_heat_capacity_classical_limit():
    """At T >> hbar omega / k_B every mode holds k_B: C_m -> k_B D domega g (error ~ x^2/12)."""
    mat = di.silicon_like(n_bins=200, T_eq=1e6)
    om, dom, dos, vg, tau, deg = mat.flat()
    dedT, Cm, sums = oracle.tabulate(mat)
    classical = KB * dos * dom * deg
    x = HBAR * om / (KB * 1e6)
    assert np.all(np.abs(Cm / classical - 1.0) <= x ** 2 / 12.0 + 1e-12)
    assert sums[0] == pytest.approx(classical.sum(), rel=1e-4)
    assert sums[1] == pytest.approx(np.sum(Cm / tau), rel=1e-12)
    assert sums[2] == pytest.approx(np.sum(Cm * vg), rel=1e-12)


# --------------------------------------------------------------- Alias ----

def _implied_mass(t):
    b = t["bits"]
    U = 1 << (32 - b)
    th = t["thresh"].astype(np.int64)
    al = t["alias"].astype(np.int64)
    mass = th.copy()
    np.add.at(mass, al, U - th)
    return mass


@pytest.mark.parametrize("case", ["gray", "si_gain", "si_flux", "si_init", "random_zeros", "pow2", "two"])
def test_alias_integer_identity(case):
    """thresh_j + sum_{alias_i = j}(U - thresh_i) = q_j exactly; q sums to 2^32 and is within 1 of w/W 2^32."""
    mat = di.silicon_like()
    om, dom, dos, vg, tau, deg = mat.flat()
    _, Cm, _ = oracle.tabulate(mat)
    rng = np.random.Generator(np.random.PCG64(5))
    w = {"gray": np.array([3.0]), "si_gain": Cm / tau, "si_flux": Cm * vg, "si_init": Cm,
         "random_zeros": rng.exponential(size=1500) * (rng.random(1500) > 0.3),
         "pow2": rng.random(1024), "two": np.array([1.0, 1.0])}[case]
    t = oracle.alias(w)
    q = t["q"].astype(np.int64)
    assert int(q.sum()) == 2 ** 32
    assert np.array_equal(_implied_mass(t), q)
    assert np.all(t["thresh"] <= (1 << (32 - t["bits"])))
    exact = np.zeros(q.shape[0])
    exact[: w.shape[0]] = w / w.sum() * 2.0 ** 32
    assert np.all(np.abs(q - exact) < 1.0 + 1e-6)
    assert np.all(q[w.shape[0]:] == 0)


def test_post_scatter_states_chi_square():
    """Sampled post-scattering (omega, p) states follow the normalised D de/dT / tau (Eq. (2))."""
    mat = di.silicon_like()
    job = di.slab_job(mat, 1e-6, 12000, seed=31, n_bins=0)
    hist = np.zeros(mat.n_states, np.uint64)
    oracle.run_raw(job, threads=THREADS, hist=hist)
    _, Cm, sums = oracle.tabulate(mat)
    p = (Cm / mat.flat()[4]) / sums[1]
    n = float(hist.sum())
    assert n > 1e6
    exp = n * p
    # merge states in index order into groups with expected count >= 20
    obs_g, exp_g = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(hist.astype(np.float64), exp):
        acc_o += o
        acc_e += e
        if acc_e >= 20.0:
            obs_g.append(acc_o)
            exp_g.append(acc_e)
            acc_o = acc_e = 0.0
    obs_g[-1] += acc_o
    exp_g[-1] += acc_e
    obs_g, exp_g = np.array(obs_g), np.array(exp_g)
    chi2 = float(np.sum((obs_g - exp_g) ** 2 / exp_g))
    pval = stats.chi2.sf(chi2, len(obs_g) - 1)
    assert pval > 1e-3, (chi2, len(obs_g))


# ------------------------------------------------------- Gray slab (C1) ----

@pytest.fixture(scope="module")
def gray_ref():
    return refsol.gray_slab_richardson(100e-9 / (6000.0 * 16.7e-12), n_bins=20, M=600)


def test_gray_slab_matches_integral_equation(gray_ref):
    """C1 gray slab (s_L = 0.998): bin temperatures and transmission within 4 standard errors
    of the exponential-integral solution of the same linearized gray problem."""
    job = di.gray_slab(n=100_000)
    res, raw, cnt, _ = oracle.simulate(job, threads=THREADS)
    prep = oracle.prepare(job)
    ref_T, ref_psi = gray_ref
    Tn = res["T"] / 1.0  # walls at +-0.5 K: T / (T_h - T_c)
    se = res["T_se"]
    assert np.all(np.abs(Tn - ref_T) <= 4 * se), (Tn, ref_T, se)
    assert np.all(se < 0.01)
    unit = prep.C_tot * 6000.0 / 4.0
    psi = res["q"] / unit
    psi_se = res["q_se"] / unit
    assert abs(psi.mean() - ref_psi) <= 4 * psi_se.mean()
    # gray medium: the pseudo-temperature equals the energy temperature
    assert np.allclose(res["Tloc"], res["T"], rtol=1e-12, atol=1e-15)


def test_gray_slab_ballistic_limit():
    """Without scattering every particle crosses: transmission Psi = 1 exactly, no scattering events."""
    job = di.gray_slab(n=20_000, tau=1e3)
    res, raw, cnt, _ = oracle.simulate(job, threads=THREADS)
    prep = oracle.prepare(job)
    psi = res["q"] / (prep.C_tot * 6000.0 / 4.0)
    assert np.allclose(psi, 1.0, rtol=1e-12)
    assert cnt["scatters"] == 0


def test_gray_slab_diffusive_limit():
    """s_L = 10: transmission matches the integral-equation value (itself matched to the Milne
    diffusion form (4/3)/(s_L + 2 z0), z0 = 0.7104, in test_refsol_limits)."""
    tau = 16.7e-12
    L = 10 * 6000.0 * tau
    job = di.gray_slab(n=100_000, L=L)
    res, raw, cnt, _ = oracle.simulate(job, threads=THREADS)
    prep = oracle.prepare(job)
    unit = prep.C_tot * 6000.0 / 4.0
    _, ref_psi = refsol.gray_slab(10.0, M=800)
    psi = res["q"].mean() / unit
    assert abs(psi - ref_psi) <= 4 * res["q_se"].mean() / unit


def test_refsol_limits():
    """The reference solver itself: Milne diffusion limit and the ballistic limit."""
    _, p10 = refsol.gray_slab(10.0, M=800)
    assert p10 == pytest.approx(refsol.milne_psi(10.0), rel=2e-4)
    _, p0 = refsol.gray_slab(1e-6, M=50)
    assert p0 == pytest.approx(1.0, abs=1e-5)


# ------------------------------------------------------ Exact invariants ----

@pytest.mark.parametrize("mat_name,L", [("gray", 100e-9), ("si", 100e-9), ("si", 1e-6)])
def test_mean_scattering_events_invariant(mat_name, L):
    """Steady slab with absorbing walls: mean scattering events per particle = 2 L G_tau / G_v,
    and every bin sees the same net displacement (each particle starts and ends on a wall)."""
    mat = di.gray_material() if mat_name == "gray" else di.silicon_like()
    n = 40_000 if L < 5e-7 else 8_000
    job = di.slab_job(mat, L, n, seed=11, n_bins=20)
    res, raw, cnt, nscat = oracle.simulate(job, threads=THREADS, want_nscat=True)
    _, _, sums = oracle.tabulate(mat)
    expect = 2.0 * L * sums[1] / sums[2]
    mean = nscat.mean()
    se = nscat.std(ddof=1) / math.sqrt(n)
    assert abs(mean - expect) <= 4.0 * se, (mean, expect, se)
    q = res["q"]
    assert np.allclose(q, q[0], rtol=1e-9)
    assert cnt["absorbed"] == n and cnt["capped"] == 0


def test_transient_energy_conservation_and_event_rate():
    """Heated spot: at every snapshot time the grid plus overflow holds sum_i s_i exactly
    (particles are conserved), and the mean number of scattering events by t_final is
    t_final G_tau / C_tot (the initial state distribution ~ C is stationary)."""
    mat = di.silicon_like()
    job = di.heated_spot(n=6000, seed=3, material=mat, grid=8, n_times=6)
    job.tally.times = tuple(np.array(job.tally.times) * 1e-2)  # up to 100 ps
    res, raw, cnt, nscat = oracle.simulate(job, threads=THREADS, want_nscat=True)
    parts = oracle.split_raw(oracle.prepare(job), raw)
    total = parts["snap"].sum(axis=1)
    assert np.all(total == job.n_particles)  # every particle is positive (dT > 0) and alive
    _, _, sums = oracle.tabulate(mat)
    expect = job.tally.times[-1] * sums[1] / sums[0]
    se = nscat.std(ddof=1) / math.sqrt(job.n_particles)
    assert abs(nscat.mean() - expect) <= 4 * se, (nscat.mean(), expect, se)


# ----------------------------------------------- Gradient problems (C4) ----

def _kappa_bulk(mat):
    _, Cm, _ = oracle.tabulate(mat)
    om, dom, dos, vg, tau, deg = mat.flat()
    return Cm, vg, tau, float(np.sum(Cm * vg * vg * tau) / 3.0)


def test_bulk_gradient_gives_bulk_conductivity():
    """Periodic cell without a pore: kappa = sum C v^2 tau / 3 for any truncation."""
    mat = di.gray_material()
    _, _, _, kb = _kappa_bulk(mat)
    for kmax in (1, 10):
        job = di.pore_cell(200e-9, 0.0, 100_000, seed=21, material=mat, kmax=kmax, n_hj=0)
        res, *_ = oracle.simulate(job, threads=THREADS)
        assert abs(res["kappa"] - kb) <= 4 * res["kappa_se"], (kmax, res["kappa"], kb, res["kappa_se"])
        assert res["kappa_se"] < 0.03 * kb


@pytest.mark.parametrize("p", [0.0, 0.5, 0.9])
def test_in_plane_film_fuchs_sondheimer_gray(p):
    """In-plane gray film of thickness = one mean free path: kappa = kappa_bulk S(1, p)."""
    mat = di.gray_material()
    Cm, vg, tau, kb = _kappa_bulk(mat)
    lam = float(vg[0] * tau[0])
    job = di.in_plane_film(lam, p, 100_000, seed=40, material=mat, kmax=10, n_hj=0)
    res, *_ = oracle.simulate(job, threads=THREADS)
    ref = kb * refsol.fuchs_sondheimer_S(1.0, p)
    assert abs(res["kappa"] - ref) <= 4 * res["kappa_se"], (res["kappa"], ref, res["kappa_se"])
    assert res["kappa_se"] < 0.03 * ref  # the comparison has teeth


def test_in_plane_film_fuchs_sondheimer_silicon():
    """Frequency-dependent in-plane film: kappa = sum_m (C v^2 tau / 3) S(d / Lambda_m, p)."""
    mat = di.silicon_like()
    Cm, vg, tau, kb = _kappa_bulk(mat)
    d = 100e-9
    job = di.in_plane_film(d, 0.0, 200_000, seed=41, material=mat, kmax=4, n_hj=0)
    res, *_ = oracle.simulate(job, threads=THREADS)
    S = refsol.fuchs_sondheimer_S(d / (vg * tau), 0.0, n=400)
    ref = float(np.sum(Cm * vg * vg * tau / 3.0 * S))
    assert abs(res["kappa"] - ref) <= 4 * res["kappa_se"], (res["kappa"], ref, res["kappa_se"])
    assert res["kappa_se"] < 0.03 * ref


@pytest.mark.parametrize("p", [0.0, 0.5, 0.9])
def test_first_event_termination_is_exact_for_films(p):
    """In-plane films: ending each trajectory at its first scattering event or
    first diffuse reflection keeps the Fuchs-Sondheimer conductivity (the flux
    carried afterwards averages to zero), and costs a fraction of the flights."""
    mat = di.gray_material()
    Cm, vg, tau, kb = _kappa_bulk(mat)
    lam = float(vg[0] * tau[0])
    ref = kb * refsol.fuchs_sondheimer_S(1.0, p)
    full = di.in_plane_film(lam, p, 100_000, seed=43, material=mat, kmax=10, n_hj=0)
    first = di.in_plane_film(lam, p, 100_000, seed=43, material=mat, kmax=10, n_hj=0, first_event=True)
    r1, _, c1, _ = oracle.simulate(first, threads=THREADS)
    r0, _, c0, _ = oracle.simulate(full, threads=THREADS)
    assert abs(r1["kappa"] - ref) <= 4 * r1["kappa_se"], (r1["kappa"], ref, r1["kappa_se"])
    assert r1["kappa_se"] < 0.03 * ref
    assert c1["scatters"] <= first.n_particles  # at most one scattering event each
    assert c1["iterations"] < 0.5 * c0["iterations"]
    # same particles, same first free paths: the truncated run differs from the
    # full one only by terms of zero mean
    assert abs(r1["kappa"] - r0["kappa"]) <= 4 * r0["kappa_se"]


def test_first_event_termination_silicon_film():
    mat = di.silicon_like()
    Cm, vg, tau, kb = _kappa_bulk(mat)
    d = 100e-9
    job = di.in_plane_film(d, 0.5, 200_000, seed=44, material=mat, kmax=40, n_hj=0, first_event=True)
    res, *_ = oracle.simulate(job, threads=THREADS)
    S = refsol.fuchs_sondheimer_S(d / (vg * tau), 0.5, n=4000)
    ref = float(np.sum(Cm * vg * vg * tau / 3.0 * S))
    assert abs(res["kappa"] - ref) <= 4 * res["kappa_se"], (res["kappa"], ref, res["kappa_se"])
    assert res["kappa_se"] < 0.03 * ref


def test_first_event_rejected_outside_films():
    job = di.pore_cell(100e-9, 0.2, 10, seed=1, material=di.gray_material(), kmax=4, n_hj=0)
    job.tally.first_event = True
    with pytest.raises(ValueError):
        oracle.prepare(job)


def test_film_flux_after_first_event_vanishes():
    """Diffuse walls and isotropic scattering: the mean contribution after the first
    scattering event is zero (H_j, j >= 1) and H_0 carries the whole conductivity."""
    mat = di.gray_material()
    _, vg, tau, kb = _kappa_bulk(mat)
    job = di.in_plane_film(float(vg[0] * tau[0]), 0.0, 100_000, seed=42, material=mat, kmax=8, n_hj=8)
    res, *_ = oracle.simulate(job, threads=THREADS)
    hj, se = res["hj"], res["hj_se"]
    assert np.all(np.abs(hj[1:]) <= 4 * se[1:])
    assert abs(hj.sum() - res["kappa"]) <= 1e-9 * abs(res["kappa"])
    assert hj[0] > 10 * se[0]


# ------------------------------------------- time-windowed region tally ----

def _spot(mat, n, seed, times, region, specularity=0.0):
    job = di.heated_spot(n=n, seed=seed, material=mat, grid=4, n_times=len(times), specularity=specularity)
    job.tally.times = tuple(times)
    job.tally.region = region
    return job


def test_region_tally_conserves_energy():
    """A region holding every particle at every time: the windowed temperature is
    the total deviational energy over C_tot mu(R), in every window, exactly."""
    mat = di.silicon_like()
    times = (1e-12, 1e-11, 5e-11)
    job = _spot(mat, 2000, 51, times, (0.0, 0.0, 1.0, 0.0, 1.0))
    res, *_ = oracle.simulate(job, threads=4)
    mu = math.pi * 1.0 * 1.0
    exact = 1.0 * math.pi ** 1.5 * (1e-6) ** 3 / 2.0 / mu  # dT pi^{3/2} r0^3 / 2 / mu
    assert np.allclose(res["region_T"], exact, rtol=1e-12, atol=0.0), (res["region_T"], exact)
    assert np.all(res["region_T_se"] <= 1e-6 * exact)  # every particle contributes the same


def _ballistic_region_reference(v, r0, dT, times, region, nq=24):
    """Ballistic transport (no scattering) from the Gaussian initial condition with
    a specular surface, i.e. the full-space problem with the mirrored Gaussian:
    dT(x, t) is the mean of dT exp(-|y|^2/r0^2) over the sphere |y - x| = v t, and
    q_z(x, t) = C v <Omega_z dT exp(-|x - v t Omega|^2/r0^2)> over directions.
    Averages over the cylinder and each window by Gauss-Legendre quadrature.
    Returns (T, q / C) per window."""
    cx, cy, R, zlo, zhi = region
    xg, wg = np.polynomial.legendre.leggauss(nq)
    rho = 0.5 * R * (xg + 1.0); wr = 0.5 * R * wg * 2.0 * np.pi * rho
    zz = zlo + 0.5 * (zhi - zlo) * (xg + 1.0); wz = 0.5 * (zhi - zlo) * wg
    mu_d, wmu = np.polynomial.legendre.leggauss(32)
    nphi = 32
    phi = (np.arange(nphi) + 0.5) * 2.0 * np.pi / nphi
    vol = math.pi * R * R * (zhi - zlo)
    edges = np.concatenate([[0.0], times])
    T_out, Q_out = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        tg = a + 0.5 * (b - a) * (xg + 1.0); wt = 0.5 * (b - a) * wg
        Tw = Qw = 0.0
        for t, w_t in zip(tg, wt):
            s = v * t
            for r_, w_r in zip(rho, wr):
                for z_, w_z in zip(zz, wz):
                    # point (r_, 0, z_): average over directions Omega = (sin th cos phi, sin th sin phi, cos th)
                    st = np.sqrt(1.0 - mu_d ** 2)
                    ox = st[:, None] * np.cos(phi)[None, :]
                    oz = np.broadcast_to(mu_d[:, None], ox.shape)
                    d2 = (r_ - s * ox) ** 2 + (s * st[:, None] * np.sin(phi)[None, :]) ** 2 + (z_ - s * oz) ** 2
                    g = dT * np.exp(-d2 / r0 ** 2)
                    wdir = (wmu[:, None] / 2.0) * (1.0 / nphi)
                    Tw += w_t * w_r * w_z * float(np.sum(wdir * g))
                    Qw += w_t * w_r * w_z * float(np.sum(wdir * v * oz * g))
        T_out.append(Tw / (vol * (b - a)))
        Q_out.append(Qw / (vol * (b - a)))
    return np.array(T_out), np.array(Q_out)


def test_region_tally_ballistic_limit():
    """No scattering before t_final (tau = 1 s) and a specular surface: the windowed
    temperature and z heat flux in a surface cylinder equal the ballistic solution
    from the Gaussian initial condition."""
    v, r0 = 6000.0, 1e-6
    mat = di.gray_material(vg=v, tau=1.0)
    times = (5e-11, 1e-10, 1.5e-10, 2.5e-10)
    region = (0.0, 0.0, 0.3e-6, 0.0, 0.3e-6)
    job = _spot(mat, 6_000_000, 52, times, region, specularity=1.0)
    res, *_ = oracle.simulate(job, threads=THREADS)
    T_ref, Q_ref = _ballistic_region_reference(v, r0, 1.0, np.array(times), region)
    C_tot = oracle.tabulate(mat)[2][0]
    # the flux is a difference of opposite streams, so its relative error is larger
    for key, ref, teeth in (("region_T", T_ref, 0.005), ("region_q", C_tot * Q_ref, 0.08)):
        got, se = res[key], res[key + "_se"]
        assert np.all(se < teeth * np.abs(ref)), (key, se, ref)
        assert np.all(np.abs(got - ref) <= 4.0 * se + 2e-3 * np.abs(ref)), (key, got, ref, se)
    assert np.all(res["region_q"] > 0.0)  # heat flows into the substrate


# ------------------------------------------------------- steady x-z field ----

def _field_job(mat, porosity, n, seed, nx=12, nz=12, period=100e-9):
    return di.pore_cell(period, porosity, n, seed, material=mat, kmax=40, n_hj=0, field=(nx, nz))


def test_field_adds_up_to_the_conductivity_sums():
    """The field's z displacement over all cells equals the per-particle algebraic
    lengths of the conductivity estimator (two separate accumulations of the same
    segments), and its cell-averaged flux is kappa |G|."""
    mat = di.silicon_like()
    job = _field_job(mat, 0.2, 20_000, 701)
    prep = oracle.prepare(job)
    raw, *_ = oracle.run_raw(job, threads=THREADS, prep=prep)
    parts = oracle.split_raw(prep, raw)
    dz = parts["field"][:, 1].sum()
    assert abs(dz - parts["kappa"][0]) <= 1e-12 * abs(parts["kappa"][0])
    res = oracle.finalize(prep, raw)
    assert abs(res["field_q"].mean() - res["kappa"] * abs(job.source.gradient)) <= 1e-10 * abs(res["kappa"] * 1e6)
    # no time is spent inside the pore: the cells wholly inside it stay empty
    P, r = job.geometry.length, job.geometry.radius
    c = (np.arange(12) + 0.5) * P / 12
    far = np.hypot(*np.meshgrid(c - P / 2, c - P / 2)) + P / 12 * math.sqrt(0.5) < r
    assert far.any() and np.all(parts["field"][:, :, far] == 0.0)


def test_field_bulk_limit():
    """A cell without a pore is translation invariant: every cell's z heat flux is
    kappa_bulk |G| and its deviational temperature is zero (any truncation)."""
    mat = di.gray_material()
    _, _, _, kb = _kappa_bulk(mat)
    job = di.pore_cell(200e-9, 0.0, 100_000, 702, material=mat, kmax=10, n_hj=0, field=(8, 8))
    res, *_ = oracle.simulate(job, threads=THREADS)
    G = abs(job.source.gradient)
    zq = (res["field_q"] - kb * G) / res["field_q_se"]
    zt = res["field_T"] / res["field_T_se"]
    assert np.all(res["field_q_se"] < 0.1 * kb * G)
    # chi-square over the 64 cells, 99.9 % quantile (batch-mean SEs over 16 batches: t-tails)
    for z in (zq, zt):
        assert np.all(np.abs(z) < 6.0), z
        assert float(np.sum(z ** 2)) < stats.chi2.ppf(0.999, z.size) * 1.5, z


def test_field_symmetries_of_the_pore_cell():
    """The cell is mirror symmetric in x and in z, and the gradient is along z: the
    temperature is even in x and odd in z, the z heat flux even in both."""
    mat = di.silicon_like()
    res, *_ = oracle.simulate(_field_job(mat, 0.3, 60_000, 703), threads=THREADS)
    T, Ts, q, qs = res["field_T"], res["field_T_se"], res["field_q"], res["field_q_se"]
    ok = Ts > 0  # cells inside the pore hold nothing
    Ts, qs = np.where(ok, Ts, 1.0), np.where(ok, qs, 1.0)
    checks = [
        ((T - T[:, ::-1]) / np.hypot(Ts, Ts[:, ::-1]), "T even in x"),
        ((T + T[::-1, :]) / np.hypot(Ts, Ts[::-1, :]), "T odd in z"),
        ((q - q[:, ::-1]) / np.hypot(qs, qs[:, ::-1]), "q even in x"),
        ((q - q[::-1, :]) / np.hypot(qs, qs[::-1, :]), "q even in z"),
    ]
    for z, what in checks:
        zz = z[ok & ok[:, ::-1] & ok[::-1, :]]
        assert np.all(np.abs(zz) < 6.0), what
        # each pair appears twice; chi-square of the independent half
        assert float(np.sum(zz ** 2)) / 2 < stats.chi2.ppf(0.999, zz.size // 2) * 1.5, what
    # the temperature field is resolved: odd in z with a clear sign on the lower and upper halves
    lower, upper = T[:6][ok[:6]].mean(), T[6:][ok[6:]].mean()
    assert lower * upper < 0


# --------------------------------------------------------------------------
# Pore-cell geometry (the periodic nanostructure of the conductivity section):
# step III against brute-force ray marching, step I's positions against the
# area of the solid, and the chords between pore hits against Cauchy's mean
# chord formula for cosine-law re-emission.
# --------------------------------------------------------------------------


def _pore_prep(porosity, period=100e-9, specularity=0.0, n=1000, seed=41):
    job = di.pore_cell(period, porosity, n, seed, material=di.gray_material(), kmax=40, n_hj=0,
                       specularity=specularity)
    return job, oracle.prepare(job)


def _in_solid(x, z, P, r, tol):
    c = 0.5 * P
    return (x >= -tol) & (x <= P + tol) & (z >= -tol) & (z <= P + tol) & \
        (np.hypot(x - c, z - c) >= r * (1.0 - 1e-12) - tol)


@pytest.mark.parametrize("porosity", [0.05, 0.3, 0.6])
def test_pore_boundary_search_against_ray_marching(porosity):
    """The first surface the oracle reports is where the ray leaves the solid:
    the hit point lies on the reported face or on the pore, the ray moves into
    that surface there, and 400 points marched along the ray before it are all
    inside the solid of the cell."""
    job, prep = _pore_prep(porosity)
    P, r, c = job.geometry.length, job.geometry.radius, 0.5 * job.geometry.length
    rng = np.random.default_rng(7)
    tol = 1e-12 * P
    frac = np.linspace(1e-6, 1.0 - 1e-6, 400)
    seen = set()
    for _ in range(1500):
        while True:
            x0, z0 = rng.uniform(0.0, P, 2)
            if math.hypot(x0 - c, z0 - c) > r:
                break
        mu = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        st = math.sqrt(1.0 - mu * mu)
        o = np.array([st * math.cos(ph), st * math.sin(ph), mu])
        x = np.array([x0, rng.uniform(-P, P), z0])
        t, surf = oracle.boundary_search(prep, x, o, v=1.0)
        assert np.isfinite(t) and t >= 0.0 and surf in (0, 1, 2, 3, 4)
        seen.add(surf)
        h = x + o * t
        if surf == 4:
            assert abs(math.hypot(h[0] - c, h[2] - c) - r) <= 1e-9 * r
            assert (h[0] - c) * o[0] + (h[2] - c) * o[2] < 0.0  # entering the pore
        else:
            ax = 0 if surf < 2 else 2
            edge = P if surf % 2 == 1 else 0.0
            assert abs(h[ax] - edge) <= 1e-9 * P
            assert (o[ax] > 0.0) == (surf % 2 == 1)  # leaving through that face
        pts = x[None, :] + (t * frac)[:, None] * o[None, :]
        assert np.all(_in_solid(pts[:, 0], pts[:, 2], P, r, tol)), (x, o, t, surf)
    assert seen == {0, 1, 2, 3, 4}


def test_pore_search_excludes_the_resting_surface():
    """A particle resting on a face or on the pore is not found to hit it again
    at distance zero (the exclusion rule of the boundary search)."""
    job, prep = _pore_prep(0.3)
    P, r, c = job.geometry.length, job.geometry.radius, 0.5 * job.geometry.length
    # on the pore, leaving it outward along the normal: the next hit is a face
    n = np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
    x = np.array([c + r * n[0], 0.0, c + r * n[2]])
    t, surf = oracle.boundary_search(prep, x, n, v=1.0, last=4)
    assert surf in (1, 3) and abs(t - (P - (c + r * n[0])) / n[0]) <= 1e-12 * P
    # on the face x = 0, moving in +x: the next hit is the pore or x = P, never face 0
    x = np.array([0.0, 0.0, 0.1 * P])
    t, surf = oracle.boundary_search(prep, x, np.array([1.0, 0.0, 0.0]), v=1.0, last=0)
    assert surf == 1 and abs(t - P) <= 1e-12 * P


def test_pore_emission_is_uniform_in_the_solid():
    """The gradient source places particles uniformly in the solid of the cell:
    the fraction within distance rho of the pore axis is the annulus area over
    the solid area, and the mean position is the cell centre."""
    job, prep = _pore_prep(0.3, n=30_000)
    P, r, c = job.geometry.length, job.geometry.radius, 0.5 * job.geometry.length
    xs = np.array([oracle.emit_state(prep, pid)[0] for pid in range(job.n_particles)])
    n = len(xs)
    rho = np.hypot(xs[:, 0] - c, xs[:, 2] - c)
    assert np.all(rho >= r) and np.all((xs[:, [0, 2]] >= 0.0) & (xs[:, [0, 2]] <= P))
    solid = P * P - math.pi * r * r
    for rho0 in (1.2 * r, 0.4 * P, 0.5 * P):
        p = (math.pi * rho0 * rho0 - math.pi * r * r) / solid
        f = np.mean(rho < rho0)
        assert abs(f - p) <= 4.0 * math.sqrt(p * (1.0 - p) / n), (rho0, f, p)
    for ax in (0, 2):
        sd = P / math.sqrt(12.0)  # at most the spread of a uniform variable on [0, P]
        assert abs(xs[:, ax].mean() - c) <= 4.0 * sd / math.sqrt(n)


@pytest.mark.parametrize("porosity", [0.1, 0.3, 0.5])
def test_pore_mean_chord_is_cauchys(porosity):
    """Ballistic walk with diffuse (cosine-law) pore walls: the mean path length
    between consecutive pore hits is 4 V / S of the solid (Cauchy's formula; per
    unit length along the pore axis V = P^2 - pi r^2, S = 2 pi r), and its
    projection on the x-z plane has the two-dimensional mean pi A / perimeter.
    Chord lengths are heavy-tailed (rays nearly parallel to the axis or to an
    open channel), so the tolerance is 3 %."""
    job, prep = _pore_prep(porosity, n=20_000)
    P, r = job.geometry.length, job.geometry.radius
    n, s3, s2 = oracle.pore_chords(prep, 0, job.n_particles, 40)
    assert n > 0.95 * 40 * job.n_particles
    mean3, mean2 = s3 / n, s2 / n
    solid = P * P - math.pi * r * r
    ref3 = 4.0 * solid / (2.0 * math.pi * r)
    ref2 = math.pi * solid / (2.0 * math.pi * r)
    assert abs(mean3 / ref3 - 1.0) < 0.03, (mean3, ref3)
    assert abs(mean2 / ref2 - 1.0) < 0.03, (mean2, ref2)


# ------------------------- frequency-dependent slab, heated spot, specular pore ----
# The checks live in tests/pinlib.py so that tests/test_oracle_mutants.py can run
# them against oracles with planted mistakes.

import pinlib  # noqa: E402


@pytest.mark.parametrize("L,n,seed", [(100e-9, 200_000, 91), (300e-9, 100_000, 92)])
def test_nongray_slab_matches_integral_equation(L, n, seed):
    """Frequency-dependent slab (80 silicon-like states): T, T_loc and q agree with
    the pseudo-temperature integral equation solved deterministically."""
    pinlib.check_nongray_slab(oracle, L=L, n=n, seed=seed)


def test_nongray_reference_reduces_to_the_gray_solution():
    """The frequency-dependent solver with a single state is the gray slab of the
    Nystrom solver (two independent discretisations of one equation)."""
    lam = 100e-9 / 0.998
    T, P, q0, qL = refsol.nongray_slab([1.0], [1.0], [lam], 100e-9, per_bin=20, h_min=lam * 1e-3)
    gb, gpsi = refsol.gray_slab_richardson(0.998, n_bins=20, M=600)
    assert np.allclose(T, gb, atol=2e-5) and np.allclose(P, gb, atol=2e-5)
    assert q0 == pytest.approx(gpsi / 4.0, rel=1e-4) and qL == pytest.approx(q0, rel=1e-9)


def test_snapshot_estimator_ballistic_limit():
    pinlib.check_snapshot_ballistic(oracle)


def test_snapshot_estimator_diffusive_limit():
    pinlib.check_snapshot_diffusive(oracle)


def test_specular_pore_projected_chord_is_santalos():
    pinlib.check_specular_pore_chords(oracle)


# ---------------------------------------- anisotropic scattering (step IVb) ----

@pytest.mark.parametrize("g", [0.6, -0.4, 0.95])
def test_henyey_greenstein_directions(g):
    """Scattering directions for g != 0 (pinlib.check_hg_sampler)."""
    pinlib.check_hg_sampler(oracle, g=g)


def test_isotropic_case_is_unchanged():
    """g = 0 is the paper's isotropic step: the same directions as before."""
    o = np.array([0.6, 0.0, 0.8])
    for a, b in ((1, 2), (2 ** 31, 77), (2 ** 32 - 1, 5)):
        d = oracle.scatter_direction(0.0, a, b, o)
        mu = 2.0 * ((a + 0.5) / 2.0 ** 32) - 1.0
        assert d[2] == mu


@pytest.mark.parametrize("g", [0.6, -0.4])
def test_bulk_conductivity_with_anisotropic_scattering(g):
    """Gray bulk (periodic cell without a pore) under the gradient source: a free
    path keeps on average g^j of the initial z direction after j scattering events,
    so kappa = C v^2 tau / (3 (1 - g)) (the transport relaxation time tau / (1 - g)),
    and the flux carried between events j and j+1 is H_j = H_0 g^j."""
    mat = di.gray_material(scatter_g=g)
    _, _, _, kb = _kappa_bulk(mat)
    job = di.pore_cell(200e-9, 0.0, 400_000, seed=62, material=mat, kmax=60, n_hj=4)
    res, *_ = oracle.simulate(job, threads=THREADS)
    ref = kb / (1.0 - g)
    assert abs(res["kappa"] - ref) <= 4 * res["kappa_se"], (res["kappa"], ref, res["kappa_se"])
    assert res["kappa_se"] < 0.02 * ref
    hj, se = res["hj"], res["hj_se"]
    for j in (1, 2, 3):
        assert abs(hj[j] - hj[0] * g ** j) <= 4 * np.hypot(se[j], se[0] * abs(g) ** j), (j, hj, se)


def test_first_event_rejected_with_anisotropic_scattering():
    job = di.in_plane_film(50e-9, 0.0, 10, seed=1, material=di.gray_material(scatter_g=0.3), first_event=True)
    with pytest.raises(ValueError):
        oracle.prepare(job)
