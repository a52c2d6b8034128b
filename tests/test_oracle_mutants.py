"""The pins can fail: each case plants one plausible mistake in a copy of the
oracle's C source (a sign, a dropped term, a swapped operand or sub-step),
builds it, and runs the oracle's pin tests against that build in a separate
process, which must then fail.  A control build of the unchanged source must
pass the same tests.  CPU only; the mistakes live in the copy, never in the
oracle itself."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_exact.py", "tests/test_oracle_dispersion.py",
        "tests/test_oracle_strang.py", "tests/test_oracle_field.py",
        "tests/test_oracle_observables_adjoint.py", "tests/test_oracle_pulse.py"]

# (name, text in dirac_oracle.c, its planted replacement, pin files that must catch it)
MUTANTS = [
    ("sigma_y sign", "{{0, -I}, {I, 0}},  /* sigma_y */", "{{0, I}, {-I, 0}},  /* sigma_y */",
     ["tests/test_oracle_dispersion.py", "tests/test_oracle_exact.py"]),
    ("projectors swapped", "PROJ[d][0][r][s] = 0.5 * (id + ALPHA[d][r][s]);",
     "PROJ[d][0][r][s] = 0.5 * (id - ALPHA[d][r][s]);", ["tests/test_oracle_exact.py"]),
    ("mass term dropped", "const double th = (v + creal(BETA[k][k]) * mc2) * dt;",
     "const double th = (v + 0.0 * creal(BETA[k][k]) * mc2) * dt;",
     ["tests/test_oracle_exact.py", "tests/test_oracle_dispersion.py"]),
    ("phase sign", "psi[4 * s + k] *= CMPLX(cos(th), sign * sin(th));",
     "psi[4 * s + k] *= CMPLX(cos(th), -sign * sin(th));",
     ["tests/test_oracle_exact.py", "tests/test_oracle_dispersion.py"]),
    ("3-D second-order sub-step", "{order[2], 2}, {-1, 0},", "{order[1], 2}, {-1, 0},",
     ["tests/test_oracle_strang.py", "tests/test_oracle_field.py"]),
    ("field coupling sign", "U[0][2] = CMPLX(0.0, az * sA);", "U[0][2] = CMPLX(0.0, -az * sA);",
     ["tests/test_oracle_field.py"]),
    ("adjoint direction", "PROJ_H[a][1], PROJ_H[a][0], lam, tmp);",
     "PROJ_H[a][0], PROJ_H[a][1], lam, tmp);", ["tests/test_oracle_observables_adjoint.py"]),
    ("cell centre", "const double x0 = xmin[0] + ((double)i0 + 0.5) * dx;",
     "const double x0 = xmin[0] + ((double)i0) * dx;", ["tests/test_oracle_observables_adjoint.py"]),
    ("pulse ramp", "if (t < t_on) return t / t_on;", "if (t < t_on) return t / pp[4];",
     ["tests/test_oracle_pulse.py"]),
    ("quadrature weight", "w[k] = 2.0 / ((1.0 - z * z) * dp * dp);",
     "w[k] = 2.0 / ((1.0 + z * z) * dp * dp);", ["tests/test_oracle_pulse.py"]),
]


def _build(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src_text)
    subprocess.run(["gcc", *O.CFLAGS, str(c), "-o", str(so), "-lm"], check=True)
    return str(so)


def _run_pins(so, files):
    env = dict(os.environ, DIRAC_ORACLE_LIB=so, DIRAC_SLOW="0")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *files], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _source():
    with open(os.path.join(ROOT, "oracle", "dirac_oracle.c")) as f:
        return f.read()


def test_control_build_passes_the_pins(tmp_path):
    so = _build(_source(), tmp_path, "control")
    rc, out = _run_pins(so, PINS)
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new,files", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, files):
    src = _source()
    assert old in src, f"mutation target missing: {old}"
    bad = src.replace(old, new, 1)
    so = _build(bad, tmp_path, "mutant")
    rc, out = _run_pins(so, files)
    assert rc == 1, f"{name}: the pins did not fail (rc {rc})\n{out}"
