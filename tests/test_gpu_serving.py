"""Continuous-batching server: requests admitted by device memory and slots,
sliced across epoch launches shared with other requests, give the same
result as when they run alone (same realisation: only the order of FP64
additions differs)."""
import numpy as np
import pytest

import dmc_inputs as di
from gpu_cases import rel_diff, small_spot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1206_3316_amd import binding as b  # noqa: E402


def _requests(si):
    return [
        di.slab_job(si, 2e-7, 30_000, seed=2001, n_bins=20),
        small_spot(n=8_000, seed=2002, grid=8, n_times=5, mat=si),
        di.pore_cell(80e-9, 0.25, 20_000, seed=2003, material=si, kmax=40, n_hj=8),
        di.slab_job(si, 1e-6, 5_000, seed=2004, n_bins=20),
        di.in_plane_film(50e-9, 0.5, 25_000, seed=2005, material=si, kmax=40, n_hj=4),
        di.slab_job(si, 3e-8, 60_000, seed=2006, n_bins=20),
        di.pore_cell(90e-9, 0.2, 15_000, seed=2009, material=si, kmax=40, n_hj=4, field=(8, 8)),
    ]


@pytest.mark.parametrize("class_epochs", [False, True])
def test_mix_equals_alone_and_requests_join_running_epochs(class_epochs):
    """Mixed epochs (every request, the generic kernel) and class epochs (each
    epoch one class of requests in its specialised kernel, the other classes'
    suspended particles waiting) both give every request its solo result."""
    si = di.silicon_like()
    mat = b.Material(si)
    reqs = _requests(si)
    # a small epoch budget slices every request over several epochs; a small memory
    # budget and 3 slots force queueing and admission as memory frees up
    srv = b.Server(mat, memory_budget=4 << 20, max_active=3, epoch_flights=1e6, class_epochs=class_epochs)
    tickets = [srv.submit(j) for j in reqs[:3]]
    srv.step()
    q, r = srv.load()
    assert r >= 1
    tickets += [srv.submit(j) for j in reqs[3:]]  # arrive while others are running
    steps = 0
    while not all(srv.done(t) for t in tickets):
        srv.step()
        steps += 1
        assert steps < 10_000
    assert steps >= 4  # every request was sliced over several epochs
    tot = srv.totals()
    assert tot.particles == sum(j.n_particles for j in reqs) and tot.kernel_ms > 0
    flights = 0
    for t, job in zip(tickets, reqs):
        res = srv.collect(t)
        solo = b.simulate([job], material=mat)
        assert rel_diff(res.raw(0), solo.raw(0)) <= 1e-12, job.name
        s1, s2 = res.stats(0), solo.stats(0)
        assert (s1.particles, s1.scatters, s1.boundary) == (s2.particles, s2.scatters, s2.boundary), job.name
        flights += s1.iterations
    assert tot.iterations == flights  # the server's totals add up its requests' counters
    assert srv.load() == (0, 0)
    srv.close()


def test_wait_runs_epochs_until_the_request_completes():
    """dmc_server_wait steps the server until one request is complete, the others
    advancing with it; each result equals its solo run, and an unknown or
    collected ticket is refused."""
    si = di.silicon_like()
    mat = b.Material(si)
    reqs = _requests(si)[:3]
    srv = b.Server(mat, memory_budget=64 << 20, max_active=3, epoch_flights=1e6)
    tickets = [srv.submit(j) for j in reqs]
    assert srv.wait(tickets[1]) >= 1
    assert srv.done(tickets[1])
    assert srv.wait(tickets[1]) == 0  # complete already: no epoch runs
    for t in tickets:
        srv.wait(t)
    for t, job in zip(tickets, reqs):
        res = srv.collect(t)
        solo = b.simulate([job], material=mat)
        assert rel_diff(res.raw(0), solo.raw(0)) <= 1e-12, job.name
    for bad in (tickets[0], 10**9):
        with pytest.raises(b.DmcError) as e:
            srv.wait(bad)
        assert e.value.code == b.DMC_E_INVALID
    assert srv.load() == (0, 0)
    srv.close()


def test_request_larger_than_budget_is_rejected():
    si = di.silicon_like()
    mat = b.Material(si)
    srv = b.Server(mat, memory_budget=64 << 10, max_active=2)
    big = di.heated_spot(n=10, seed=1, material=si, grid=32, n_times=10)
    with pytest.raises(b.DmcError):
        srv.submit(big)
    srv.close()


def test_suspend_resume_is_exact_against_oracle():
    """FP64 epochs that suspend particles after 16 flights and resume them in
    later epochs reproduce the FP64 oracle's tallies (same realisation)."""
    import oracle
    from gpu_cases import compare_sections, lib_sections, vmax_of

    si = di.silicon_like()
    mat = b.Material(si)
    jobs = [di.slab_job(si, 1e-6, 3_000, seed=2101, n_bins=20),
            di.pore_cell(100e-9, 0.3, 4_000, seed=2102, material=si, kmax=40, n_hj=10),
            small_spot(n=2_000, seed=2103, grid=8, n_times=5, mat=si)]
    srv = b.Server(mat, memory_budget=16 << 20, max_active=4, epoch_flights=2e5, drain_flights=16, precision="fp64")
    tickets = [srv.submit(j) for j in jobs]
    steps = 0
    while not all(srv.done(t) for t in tickets):
        srv.step()
        steps += 1
        assert steps < 100_000
    assert steps > 10
    for t, job in zip(tickets, jobs):
        res = srv.collect(t)
        prep = oracle.prepare(job)
        oraw, ocnt, _ = oracle.run_raw(job, threads=16, prep=prep)
        worst, ok = compare_sections(lib_sections(job, res.raw(0)), oracle.split_raw(prep, oraw), 1e-9, vmax_of(job))
        assert ok, (job.name, worst)
        st = res.stats(0)
        assert st.particles == job.n_particles and st.scatters == ocnt["scatters"], job.name
    srv.close()


def test_results_collected_between_epochs():
    """Each request is collected (and its result freed) in the step where it
    completes, while the others keep running with suspended particles: the
    server must not consult a collected request when it maps the particles that
    resume in the next epoch."""
    si = di.silicon_like()
    mat = b.Material(si)
    reqs = _requests(si) + [di.slab_job(si, 5e-7, 40_000, seed=2007, n_bins=20),
                            small_spot(n=12_000, seed=2008, grid=8, n_times=5, mat=si)]
    srv = b.Server(mat, memory_budget=8 << 20, max_active=4, epoch_flights=2e6, drain_flights=64)
    tickets = {srv.submit(j): j for j in reqs}
    left = dict(tickets)
    steps = 0
    while left:
        srv.step()
        steps += 1
        assert steps < 10_000
        for t in [t for t in left if srv.done(t)]:
            job = left.pop(t)
            res = srv.collect(t)
            solo = b.simulate([job], material=mat)
            assert rel_diff(res.raw(0), solo.raw(0)) <= 1e-12, job.name
            res.close()
            solo.close()
    assert steps >= 4
    assert srv.load() == (0, 0)
    srv.close()


@pytest.mark.parametrize("kind", ["slab", "pore", "spot"])
def test_single_class_epochs_match_oracle(kind):
    """Epochs whose requests are all of one class run that class's specialised
    kernel in its time-bounded form; FP64 epochs that suspend particles after 16
    flights reproduce the FP64 oracle (same realisation)."""
    import oracle
    from gpu_cases import compare_sections, lib_sections, vmax_of

    si = di.silicon_like()
    mat = b.Material(si)
    jobs = {
        "slab": [di.slab_job(si, 1e-6, 2_000, seed=2201, n_bins=20), di.slab_job(si, 3e-7, 3_000, seed=2202, n_bins=10)],
        "pore": [di.pore_cell(100e-9, 0.3, 3_000, seed=2203, material=si, kmax=40, n_hj=10),
                 di.in_plane_film(60e-9, 0.5, 3_000, seed=2204, material=si, kmax=40, n_hj=4)],
        "spot": [small_spot(n=1_500, seed=2205, grid=8, n_times=5, mat=si),
                 small_spot(n=1_000, seed=2206, grid=8, n_times=4, mat=si)],
    }[kind]
    srv = b.Server(mat, memory_budget=16 << 20, max_active=4, epoch_flights=2e3, drain_flights=16, precision="fp64")
    tickets = [srv.submit(j) for j in jobs]
    steps = 0
    while not all(srv.done(t) for t in tickets):
        srv.step()
        steps += 1
        assert steps < 100_000
    assert steps > 5  # every request was sliced over several epochs
    for t, job in zip(tickets, jobs):
        res = srv.collect(t)
        prep = oracle.prepare(job)
        oraw, ocnt, _ = oracle.run_raw(job, threads=16, prep=prep)
        worst, ok = compare_sections(lib_sections(job, res.raw(0)), oracle.split_raw(prep, oraw), 1e-9, vmax_of(job))
        assert ok, (job.name, worst)
        st = res.stats(0)
        assert st.particles == job.n_particles and st.scatters == ocnt["scatters"], job.name
    srv.close()
