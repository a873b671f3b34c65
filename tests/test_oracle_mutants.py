"""The oracle's pins must catch plausible mistakes (no GPU).

Each case plants one mistake in a copy of oracle/lbo.c (a textual
substitution, compiled to a temporary library), runs the named pins against
that library in a child process (LBO_LIB) and requires them to FAIL.  The
unaltered oracle passes the same pins in the rest of the suite.  Nothing here
changes oracle/ itself.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbo.c")
OBL = "tests/test_oracle_observables.py::test_nci_probe_oblique_golden"
UNI = "tests/test_oracle_observables.py::test_observables_uniform_forced_box"

# (name, original text, planted text, pins that must fail)
MUTANTS = [
    ("probe_truncates", "(int)round(v)", "(int)trunc(v)", [OBL]),
    ("probe_rounds_half_to_even", "(int)round(v)", "(int)nearbyint(v)", [OBL + "[tie_hit2]"]),
    ("probe_floors", "(int)round(v)", "(int)floor(v)", [OBL + "[a12n_hit3]"]),
    ("probe_strict_compare", "py >= psi[self]", "py > psi[self]", [OBL + "[d45_hit4_eq]"]),
    ("Q_divided_by_N", "out[5] /= p->nx;", "out[5] /= (double)h->N;", [UNI]),
    ("Q_without_half_force", "ux = (j[0] + 0.5 * F[0]) / rho;", "ux = j[0] / rho;", [UNI]),
    ("Q_d_weighted_by_rho2", "out[6] += r1 / rho * ux;", "out[6] += r2 / rho * ux;", [UNI]),
    ("momentum_without_half_force", "double ph = j[a] + 0.5 * F[a];", "double ph = j[a];", [UNI]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    mut = tmp_path / "lbo_mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "liblbo_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, LBO_LIB=str(lib), OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"{name}: pins did not fail\n{r.stdout[-2000:]}\n{r.stderr[-2000:]}"
    assert "failed" in r.stdout
