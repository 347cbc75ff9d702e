"""The batched launch for callers that cannot allocate (dmc_simulate_batch_noalloc)
against dmc_simulate_batch, through the C ABI: the same raw tallies and counters,
on two calls in a row whose second is smaller (stale contents of the shared
device scratch array would show), in FP64 and FP32."""
import numpy as np
import pytest

import dmc_inputs as di

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_cases import rel_diff, small_spot  # noqa: E402
from paper_1206_3316_amd import binding as b  # noqa: E402


def _large(si):
    return [di.slab_job(si, 10e-9, 40_000, seed=901, n_bins=20),
            di.slab_job(si, 500e-9, 8_000, seed=902, n_bins=20),
            di.in_plane_film(60e-9, 0.5, 20_000, seed=903, material=si, kmax=40, n_hj=8),
            di.pore_cell(100e-9, 0.3, 20_000, seed=904, material=si, kmax=40, n_hj=8, field=(12, 10)),
            small_spot(n=5000, seed=905, grid=16, n_times=8)]


def _small(si):
    return [di.slab_job(si, 40e-9, 3_000, seed=911, n_bins=10),
            di.pore_cell(70e-9, 0.2, 2_000, seed=912, material=si, kmax=20, n_hj=4)]


def _run_and_compare(jobs, mat, precision):
    offs = b.noalloc_offsets(jobs, mat)
    raw = torch.full((offs[-1],), float("nan"), dtype=torch.float64, device="cuda")
    cnt = torch.full((6 * len(jobs),), -1, dtype=torch.int64, device="cuda")
    print(f"no-alloc launch: {len(jobs)} jobs, {offs[-1]} doubles, {precision}", flush=True)
    got_offs = b.simulate_noalloc(jobs, raw, cnt, material=mat, precision=precision)
    assert got_offs == offs
    torch.cuda.synchronize()
    ref = b.simulate(jobs, material=mat, precision=precision)
    r = raw.cpu().numpy()
    c = cnt.cpu().numpy().reshape(-1, 6)
    for j, job in enumerate(jobs):
        a, e = r[offs[j]:offs[j + 1]], ref.raw(j)
        assert a.shape == e.shape and np.all(np.isfinite(a)), job.name
        assert rel_diff(a, e) <= 1e-12, (job.name, rel_diff(a, e))
        st = ref.stats(j)
        assert tuple(int(x) for x in c[j]) == (st.particles, st.scatters, st.boundary, st.iterations, st.capped,
                                               st.flights), job.name
    ref.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_no_alloc_launch_equals_the_batch_on_two_calls(precision):
    si = di.silicon_like()
    mat = b.Material(si)
    _run_and_compare(_large(si), mat, precision)
    _run_and_compare(_small(si), mat, precision)


def test_no_alloc_launch_rejects_what_does_not_fit():
    si = di.silicon_like()
    mat = b.Material(si)
    big = di.heated_spot(n=1000, seed=3, material=si)  # 64^3 cells x 50 times: 210 MB of tallies
    with pytest.raises(b.DmcError, match="at most"):
        b.noalloc_offsets([big], mat)
    many = [di.slab_job(si, 100e-9, 10, seed=i) for i in range(65)]
    with pytest.raises(b.DmcError, match="1..64"):
        b.noalloc_offsets(many, mat)
    job = di.slab_job(si, 100e-9, 1000, seed=5)
    offs = b.noalloc_offsets([job], mat)
    short = torch.zeros(offs[-1] - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(b.DmcError, match="raw_out"):
        b.simulate_noalloc([job], short, material=mat)
