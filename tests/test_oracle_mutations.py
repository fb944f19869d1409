"""The step-control pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of oracle/rkc_oracle.c (a
text substitution of one expression), builds it with the oracle's own
compiler flags, and runs the pins of tests/test_oracle_controller.py against
that library; at least one pin must fail.  The oracle itself is untouched.
"""
import concurrent.futures as cf
import functools
import os
import shutil
import subprocess
import tempfile
import types

import pytest

from oracle import build as oracle_build
from oracle import oracle as O
from tests import test_oracle_controller as C

# (name, original text, planted text); every original occurs exactly once
MUTATIONS = [
    ("RKC predictive exponent of err_{n+1}", "pow(err, -2.0 / 3.0)", "pow(err, -1.0 / 2.0)"),
    ("RKC predictive exponent of err_n", "pow(err_prev, 1.0 / 3.0)", "pow(err_prev, 1.0 / 2.0)"),
    ("RKC non-predictive exponent", "else if (!predictive) fac = 0.8 * pow(err, -1.0 / 3.0);",
     "else if (!predictive) fac = 0.8 * pow(err, -1.0 / 2.0);"),
    ("RKC safety factor 0.9", "else fac = 0.8 * (h / h_prev)", "else fac = 0.9 * (h / h_prev)"),
    ("RKC growth limit 5", "if (fac > 10.0) fac = 10.0;", "if (fac > 5.0) fac = 5.0;"),
    ("RKC rejection factor", "double fac = isfinite(err) ? 0.8 * pow(err, -1.0 / 3.0) : 0.1;",
     "double fac = isfinite(err) ? 0.8 * pow(err, -1.0 / 2.0) : 0.1;"),
    ("initial step factor 0.2", "0.1 * ht / sqrt(e0)", "0.2 * ht / sqrt(e0)"),
    ("initial step without square root", "0.1 * ht / sqrt(e0)", "0.1 * ht / e0"),
    ("tentative step 2/sigma", "double ht = (sigma > 0.0) ? 1.0 / sigma : t_end;",
     "double ht = (sigma > 0.0) ? 2.0 / sigma : t_end;"),
    ("initial error weights from the tentative state",
     "double e0 = rms_err(del, y, y, rtol, atol, N);",
     "double e0 = rms_err(del, z, z, rtol, atol, N);"),
    ("power method safety factor 1.0", "return 1.2 * sigma;", "return 1.0 * sigma;"),
    ("power method stopping test 5 %", "fabs(sigma - sigma_prev) <= 0.01 * sigma",
     "fabs(sigma - sigma_prev) <= 0.05 * sigma"),
    ("power method cap 40", "if (k == 50) break;", "if (k == 40) break;"),
    ("power method without warm start", "for (int i = 0; i < N; ++i) v[i] = z[i] - y[i];",
     "(void)0;"),
    ("spectral radius every 20 steps", "need_sigma = (since_sigma >= 25);",
     "need_sigma = (since_sigma >= 20);"),
    ("no spectral radius after a rejection", "need_sigma = 1;", "need_sigma = 0;"),
    ("stage-count constant 1.0", "sqrt(1.0 + 1.54 * h * sigma)", "sqrt(1.0 + 1.0 * h * sigma)"),
    ("stage count rounded", "int s = 1 + (int)floor(sqrt(1.0 + 1.54 * h * sigma));",
     "int s = 1 + (int)round(sqrt(1.0 + 1.54 * h * sigma));"),
    ("error estimate 1/2 h (f_n + f_n+1)", "0.4 * h * (f0[i] + f1[i])",
     "0.5 * h * (f0[i] + f1[i])"),
    ("RMS over N - 1", "return sqrt(s / (double)N);", "return sqrt(s / (double)(N - 1));"),
    ("error weights from y_n only", "double m1 = fabs(y1[i]);", "double m1 = fabs(y0[i]);"),
    ("RKCK growth exponent 1/4", "(errmax == 0.0) ? 5.0 : 0.9 * pow(errmax, -0.2)",
     "(errmax == 0.0) ? 5.0 : 0.9 * pow(errmax, -0.25)"),
    ("RKCK shrink exponent 1/5", "isfinite(errmax) ? 0.9 * pow(errmax, -0.25) : 0.1",
     "isfinite(errmax) ? 0.9 * pow(errmax, -0.2) : 0.1"),
    ("RKCK first trial step dt/2", "double t = 0.0, h = dt;", "double t = 0.0, h = 0.5 * dt;"),
    ("RKCK scale without |h f|", "fabs(y[i]) + fabs(k[i]) + 1e-30", "fabs(y[i]) + 1e-30"),
    ("RKCK scale without delta", "fabs(y[i]) + fabs(k[i]) + 1e-30", "fabs(y[i]) + fabs(k[i])"),
]


def _build_variant(tmp, i, orig, new):
    src = open(oracle_build.SRC).read()
    assert src.count(orig) == 1, orig
    path = os.path.join(tmp, "m%d.c" % i)
    with open(path, "w") as fh:
        fh.write(src.replace(orig, new))
    lib = os.path.join(tmp, "libm%d.so" % i)
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-pthread", "-w", "-o", lib, path, "-lm"], check=True)
    return lib


def _pins():
    """Every test of the controller module with its parameter sets expanded."""
    out = []
    for name in sorted(dir(C)):
        fn = getattr(C, name)
        if not (name.startswith("test_") and callable(fn)):
            continue
        cases = [{}]
        for mark in getattr(fn, "pytestmark", []):
            if mark.name != "parametrize":
                continue
            names = [x.strip() for x in mark.args[0].split(",")]
            vals = mark.args[1]
            cases = [dict(c, **dict(zip(names, v if len(names) > 1 else (v,))))
                     for c in cases for v in vals]
        out += [(name, functools.partial(fn, **c)) for c in cases]
    return out


@pytest.fixture(scope="module")
def variants():
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        libs = list(ex.map(lambda a: _build_variant(tmp, *a),
                           [(i, m[1], m[2]) for i, m in enumerate(MUTATIONS)]))
    yield dict(zip([m[0] for m in MUTATIONS], libs))
    shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_oracle_passes_every_pin():
    for name, pin in _pins():
        pin()


@pytest.mark.parametrize("mutation", [m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(variants, mutation, monkeypatch):
    L = O.load_variant(variants[mutation])
    shim = types.SimpleNamespace(**{k: getattr(O, k) for k in dir(O) if not k.startswith("__")})
    shim.Model = functools.partial(O.Model, library=L)
    monkeypatch.setattr(C, "O", shim)
    caught = []
    for name, pin in _pins():
        try:
            pin()
        except AssertionError:
            caught.append(name)
            break
    assert caught, "no pin fails with: " + mutation
