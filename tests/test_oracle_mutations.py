"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin tests against that
copy; at least one pin must fail.  The unmodified copy must pass.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_pins.py", "tests/test_interp_oracle.py", "tests/test_drops_oracle.py"]
SOURCES = ["ch_oracle.c", "interp_oracle.c", "drops_oracle.c"]

# (name, file, original text, planted mistake)
MUTATIONS = [
    ("weno-smoothness-coefficient", "ch_oracle.c",
     "double s0 = 13.0 / 12.0 * (a - 2.0 * b + c)", "double s0 = 12.0 / 12.0 * (a - 2.0 * b + c)"),
    ("weno-linear-weight", "ch_oracle.c",
     "double w1 = 0.6 /", "double w1 = 0.5 /"),
    ("weno-weight-power", "ch_oracle.c",
     "double w2 = 0.3 / ((eps + s2) * (eps + s2));", "double w2 = 0.3 / (eps + s2);"),
    ("weno-derivative-term", "ch_oracle.c",
     "+ 0.25 * (b - d) * (b - d);", "+ 0.5 * (b - d) * (b - d);"),
    ("weno-candidate", "ch_oracle.c",
     "double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;", "double q1 = (-b + 5.0 * c + 2.0 * d) / 6.5;"),
    ("upwind-side", "ch_oracle.c",
     "if (U >= 0.0) return oracle_weno5", "if (U <= 0.0) return oracle_weno5"),
    ("advection-sign", "ch_oracle.c",
     "E[p] = -adv[p] + lap[p] / Pe", "E[p] = adv[p] + lap[p] / Pe"),
    ("laplacian-scale", "ch_oracle.c",
     "s += (mp - 2.0 * mu0 + mm) / (h * h);", "s += (mp - 2.0 * mu0 + mm) / (h);"),
    ("biharmonic-centre", "ch_oracle.c",
     "const double row[5] = {1.0, -4.0, 6.0, -4.0, 1.0};\n    double scale = kappa",
     "const double row[5] = {1.0, -4.0, 5.0, -4.0, 1.0};\n    double scale = kappa"),
    ("cn-half-factor", "ch_oracle.c",
     "(2.0 * Pe * h * h * h * h)", "(1.0 * Pe * h * h * h * h)"),
    ("rk3-constant", "ch_oracle.c",
     "-17.0 / 60.0", "-15.0 / 60.0"),
    ("rk3-history", "ch_oracle.c",
     "RK_RHO[k] * Eold[p])", "RK_RHO[k] * E[p])"),
    ("noflux-reflection", "ch_oracle.c",
     "return m < n ? m : p - 1 - m;", "return m < n ? m : p - 2 - m;"),
    ("periodic-corner", "ch_oracle.c",
     "s->V[(size_t)c * n + col] += val;", "s->V[(size_t)c * n + col] += 0.5 * val;"),
    ("mass-volume", "ch_oracle.c",
     "return h * h * h * pairwise_sum(C, count);", "return h * h * pairwise_sum(C, count);"),
    ("hermite-slope", "interp_oracle.c",
     "double g1 = D / (x[2] - x[0]);", "double g1 = D / (x[2] - x[1]);"),
    ("odd-reflection", "interp_oracle.c",
     "if (m < 0) { *idx = -m; *sign = -1.0;", "if (m < 0) { *idx = -m; *sign = 1.0;"),
    ("solenoidal-inclusive-integration", "interp_oracle.c",
     "uf[r + i] = ref[k * nfy + j] + hx * acc;\n                acc += G[r + i];",
     "acc += G[r + i];\n                uf[r + i] = ref[k * nfy + j] + hx * acc;"),
    ("solenoidal-uniform-dz", "interp_oracle.c",
     "/ (zf[k + 1] - zf[k]);", "* ncz;"),
    ("solenoidal-gradient-sign", "interp_oracle.c",
     "(vc[(k * ncy + (j + 1) % ncy) * ncx + i] - vc[(k * ncy + j) * ncx + i]) * ncy;",
     "(vc[(k * ncy + j) * ncx + i] - vc[(k * ncy + (j + 1) % ncy) * ncx + i]) * ncy;"),
    ("solenoidal-reference-plane", "interp_oracle.c",
     "interp_component(au, uc, 1, zero1, nfy, m.fyc, nfz, m.fzc, ref);",
     "interp_component(ac, uc, 1, zero1, nfy, m.fyc, nfz, m.fzc, ref);"),
    ("drops-wall-wraps", "drops_oracle.c",
     "if (bc[d] != 0) continue;", "if (bc[d] != 0 && d == 0) continue;"),
    ("drops-threshold-strict", "drops_oracle.c",
     "if (C[nb] >= thr) {", "if (C[nb] > thr) {"),
    ("drops-one-direction", "drops_oracle.c",
     "for (int s = -1; s <= 1; s += 2) {", "for (int s = 1; s <= 1; s += 2) {"),
    ("projection-wall-continuation", "interp_oracle.c",
     "{m.nfz, m.fzc, 1.0, AX_WALL_EVEN}};\n    interp_component(af",
     "{m.nfz, m.fzc, 1.0, AX_PERIODIC}};\n    interp_component(af"),
]


def _build_and_run(tmp, edits):
    srcs = []
    for name in SOURCES:
        text = open(os.path.join(ORACLE, name)).read()
        for fname, old, new in edits:
            if fname == name:
                assert text.count(old) >= 1, old
                text = text.replace(old, new, 1)
        path = os.path.join(tmp, name)
        open(path, "w").write(text)
        srcs.append(path)
    so = os.path.join(tmp, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so]
                   + srcs + ["-lm"], check=True)
    env = dict(os.environ, CH_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + PINS, cwd=ROOT, env=env, capture_output=True, text=True)
    return r.returncode


def test_unmodified_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        assert _build_and_run(tmp, []) == 0


@pytest.mark.parametrize("name,fname,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, fname, old, new):
    with tempfile.TemporaryDirectory() as tmp:
        assert _build_and_run(tmp, [(fname, old, new)]) != 0, name


# mistakes planted in the numpy pressure oracle (oracle/pressure.py): the
# module is re-executed from the mutated source before its pins run
PY_MUTATIONS = [
    ("pressure-extrapolation", "Phat = 2.0 * P - Pold", "Phat = 2.0 * P + Pold"),
    ("pressure-face-pair", "return 0.5 * (a + np.roll(a, 1, axis=axis))",
     "return 0.5 * (a + np.roll(a, -1, axis=axis))"),
    ("pressure-split-coefficient", "(1.0 - rho2 / r) * g", "(1.0 - r / rho2) * g"),
    ("pressure-update-coefficient", "(1.0 / r - 1.0 / rho2) * gp", "(1.0 / rho2 - 1.0 / r) * gp"),
    ("pressure-neumann-ends", "T[0, 0] = T[-1, -1] = -1.0 / h ** 2",
     "T[0, 0] = T[-1, -1] = -2.0 / h ** 2"),
    ("pressure-no-clip", "np.clip(C, 0.0, 1.0)", "C"),
]

_PY_RUNNER = """
import sys
sys.path.insert(0, {root!r})
import oracle.pressure as m
path = m.__file__
src = open(path).read()
assert src.count({old!r}) >= 1
exec(compile(src.replace({old!r}, {new!r}, 1), path, "exec"), m.__dict__)
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", "tests/test_pressure_oracle.py"]))
"""


@pytest.mark.parametrize("name,old,new", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_planted_mistake_in_the_pressure_oracle_is_caught(name, old, new):
    code = _PY_RUNNER.format(root=ROOT, old=old, new=new)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 1, (name, r.stdout[-2000:], r.stderr[-2000:])


def test_unmodified_pressure_oracle_passes_through_the_runner():
    code = _PY_RUNNER.format(root=ROOT, old="import numpy as np", new="import numpy as np")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
