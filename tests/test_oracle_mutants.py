"""Planted mistakes in the oracle must fail its pins.

Each case copies the oracle (C source and Python layer) into a temporary
package, plants one plausible mistake by replacing one expression, builds it,
and runs the pin checks of tests/pinlib.py against it in a separate process
(a wrong oracle must not share the test process's loaded library).  The case
passes when at least one of the named checks fails.  This is how the pins are
shown to have teeth: each planted mistake is one that the FP64 parity with the
GPU path could not see, since both sides follow the same written steps.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))

# (name, file, original, planted, checks that must catch it)
MUTANTS = [
    ("snapshot cell index with x and y transposed", "dmc_oracle.c",
     "int64_t cell = inside ? (idx[2] * P->grid[1] + idx[1]) * P->grid[0] + idx[0] : ncell;",
     "int64_t cell = inside ? (idx[2] * P->grid[1] + idx[0]) * P->grid[0] + idx[1] : ncell;",
     ["check_snapshot_ballistic"]),
    ("snapshot position interpolated from the end of the segment", "dmc_oracle.c",
     "double dt = tj - ta;", "double dt = tb - tj;", ["check_snapshot_ballistic"]),
    ("snapshot cell volume from the x width alone", "__init__.py",
     "vcell = float(np.prod((np.array(tl.grid_hi) - np.array(tl.grid_lo)) / g))",
     "vcell = float(((tl.grid_hi[0] - tl.grid_lo[0]) / g[0]) ** 3)", ["check_snapshot_ballistic"]),
    ("pseudo-temperature weighted with the post-scattering relaxation time", "dmc_oracle.c",
     "score_bins(P, tally + lay.bins, bt, &p, v, tau_m, seg);",
     "score_bins(P, tally + lay.bins, bt, &p, v, P->tau[alias_draw(w[1], P->gain_bits, P->gain_thresh, "
     "P->gain_alias)], seg);", ["check_nongray_slab"]),
    ("wall emission weighted by C instead of C v", "dmc_oracle.c",
     "p->m = alias_draw(a[1], P->flux_bits, P->flux_thresh, P->flux_alias);",
     "p->m = alias_draw(a[1], P->init_bits, P->init_thresh, P->init_alias);", ["check_nongray_slab"]),
    ("Lambertian wall law without the square root", "dmc_oracle.c",
     "double mu = sqrt(unif(w2));", "double mu = unif(w2);", ["check_nongray_slab"]),
    ("scattering into the forward hemisphere only", "dmc_oracle.c",
     "double mu = 2.0 * unif(w2) - 1.0;", "double mu = unif(w2);", ["check_snapshot_diffusive"]),
    ("specular pore reflection removing the normal component once", "dmc_oracle.c",
     "for (int i = 0; i < 3; ++i) p->o[i] -= 2.0 * dn * n[i];",
     "for (int i = 0; i < 3; ++i) p->o[i] -= dn * n[i];", ["check_specular_pore_chords"]),
    ("pore normal taken from the cell corner instead of the pore axis", "dmc_oracle.c",
     "double nx = p->x[0] - c, nz = p->x[2] - c;", "double nx = p->x[0], nz = p->x[2];",
     ["check_specular_pore_chords"]),
    ("Henyey-Greenstein cosine with the sign of g reversed", "dmc_oracle.c",
     "double mu = (1.0 + g * g - f * f) / (2.0 * g);", "double mu = (1.0 + g * g - f * f) / (-2.0 * g);",
     ["check_hg_bulk"]),
    ("scattering frame vector t1 left unnormalised", "dmc_oracle.c",
     "double t1[3] = {n[0] * n[2] / s, n[1] * n[2] / s, -s};", "double t1[3] = {n[0] * n[2], n[1] * n[2], -s};",
     ["check_hg_sampler"]),
]

SCRIPT = """
import sys
sys.path[:0] = [{pkg!r}, {root!r}, {here!r}]
import oracle
assert oracle.__file__.startswith({pkg!r}), oracle.__file__
oracle.build(force=True)
import pinlib
failed = []
for name in {checks!r}:
    try:
        getattr(pinlib, name)(oracle)
    except AssertionError as e:
        failed.append(name)
        print("FAILED", name, str(e)[:300])
print("RESULT", ",".join(failed) if failed else "none")
"""


@pytest.mark.parametrize("name,fname,orig,planted,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, fname, orig, planted, checks):
    pkg = tmp_path / "mut"
    dst = pkg / "oracle"
    dst.mkdir(parents=True)
    for f in ("__init__.py", "dmc_oracle.c"):
        shutil.copy(os.path.join(ROOT, "oracle", f), dst / f)
    text = (dst / fname).read_text()
    assert text.count(orig) >= 1, f"mutation site not found: {orig}"
    (dst / fname).write_text(text.replace(orig, planted, 1))
    script = SCRIPT.format(pkg=str(pkg), root=ROOT, here=HERE, checks=checks)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    result = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT")][-1].split(" ", 1)[1]
    assert result != "none", f"planted mistake '{name}' passed every check: {out[-2000:]}"
