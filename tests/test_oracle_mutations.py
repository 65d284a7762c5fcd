"""The oracle's pins against planted mistakes: copies of the oracle's C
source, each with one plausible slip (a dropped factor, a wrong sign or
index, a transposed operand, a wrong pivot rule), are built on the CPU and
loaded in a child process in place of the oracle (ORACLE_LIB); its pin tests
(tests/test_oracle.py, tests/test_workload.py) must fail on every one.  The
mistakes are planted only in these temporary copies."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BODY = "bicgstab_body.h"
MAIN = "oracle.c"

# (name, file, original text, planted text)
MUTANTS = [
    ("beta without alpha/omega", BODY, "REAL beta = (rho / rho_prev) * (alpha / omega);", "REAL beta = (rho / rho_prev);"),
    ("p update sign", BODY, "p[i] = r[i] + beta * (p[i] - omega * v[i]);", "p[i] = r[i] + beta * (p[i] + omega * v[i]);"),
    ("s update sign", BODY, "s[i] = r[i] - alpha * v[i];", "s[i] = r[i] + alpha * v[i];"),
    ("x update skips the preconditioner", BODY, "x[i] = x[i] + alpha * ph[i] + omega * sh[i];",
     "x[i] = x[i] + alpha * ph[i] + omega * s[i];"),
    ("omega from (t, r)", BODY, "omega = FN(dot_)(n, t, s) / tau;", "omega = FN(dot_)(n, t, r) / tau;"),
    ("rho_prev never updated", BODY, "      rho_prev = rho;\n", "\n"),
    ("true residual sign", BODY, "    for (int i = 0; i < n; ++i) rt[i] = b[i] - rt[i];\n    res =",
     "    for (int i = 0; i < n; ++i) rt[i] = b[i] + rt[i];\n    res ="),
    ("Jacobi multiplies by the diagonal", BODY, "dinv[i] = (REAL)1 / d;", "dinv[i] = d;"),
    ("ILU(0) multiplier not divided by the pivot", BODY, "F[pk] = F[pk] / F[diag[k]];", "F[pk] = F[pk];"),
    ("ILU(0) update sign", BODY, "F[pj] = F[pj] - F[pk] * F[q];", "F[pj] = F[pj] + F[pk] * F[q];"),
    ("A = I + gamma J", MAIN, "A[k] = (ci[k] == i ? 1.0 : 0.0) - gamma * J[k];",
     "A[k] = (ci[k] == i ? 1.0 : 0.0) + gamma * J[k];"),
    ("LU pivots on the smallest entry", MAIN, "if (m > best) { best = m; p = i; }", "if (m < best) { best = m; p = i; }"),
    ("adjoint gradient transposed", MAIN, "grad_A[c * nnz + k] = -lam[i] * xc[ci[k]];",
     "grad_A[c * nnz + k] = -lam[ci[k]] * xc[i];"),
    ("assembly drops the factor 2 of A + A", MAIN, "dw[0] = 2.0 * (kr * yc[a]);", "dw[0] = (kr * yc[a]);"),
]


def _mutant_lib(tmp, idx, fname, old, new):
    d = os.path.join(tmp, f"m{idx}")
    os.makedirs(d, exist_ok=True)
    for f in (BODY, MAIN):
        shutil.copy(os.path.join(ROOT, "oracle", f), os.path.join(d, f))
    path = os.path.join(d, fname)
    text = open(path).read()
    assert text.count(old) == 1, (fname, old)
    open(path, "w").write(text.replace(old, new))
    lib = os.path.join(d, "liboracle_mut.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", lib,
                    os.path.join(d, MAIN), "-lm"], check=True, cwd=d)
    return lib


def _pins_fail(lib):
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle.py")], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=900)
    return r.returncode != 0, (r.stdout + r.stderr)[-800:]


def test_every_planted_mistake_is_caught(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    libs = [_mutant_lib(str(tmp_path), i, f, o, n) for i, (_, f, o, n) in enumerate(MUTANTS)]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_pins_fail, libs))
    missed = [MUTANTS[i][0] for i, (caught, _) in enumerate(results) if not caught]
    assert not missed, f"pins did not catch: {missed}"


def test_the_unmutated_copy_passes(tmp_path):
    """Control: the same build path with no mistake passes the pins."""
    d = tmp_path / "clean"
    d.mkdir()
    for f in (BODY, MAIN):
        shutil.copy(os.path.join(ROOT, "oracle", f), d / f)
    lib = str(d / "liboracle_clean.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", lib,
                    str(d / MAIN), "-lm"], check=True, cwd=str(d))
    failed, out = _pins_fail(lib)
    assert not failed, out
