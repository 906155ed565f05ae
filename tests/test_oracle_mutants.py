"""The oracle's pins catch plausible mistakes.

Each case copies the oracle (its C stepper and its Python readings), the
input generators and the pin tests into a temporary tree, plants one
mistake in the copy -- a dropped term, a wrong sign, index or spacing, a
transposed weight, a missing rotation -- builds it, and runs the pins
against it in a fresh interpreter: at least one pin must fail.  The
unmutated copy must pass them all.  The oracle itself is never modified.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C = "fd_oracle.c"
PY = "__init__.py"

# (name, file, text in the oracle, planted replacement); each text occurs once
MUTANTS = [
    ("laplacian: neighbour difference instead of sum", C,
     "s += c[j] * (up + dn);", "s += c[j] * (up - dn);"),
    ("laplacian: first axis's spacing on every axis", C,
     "acc += ih2[a] * s;", "acc += ih2[0] * s;"),
    ("leapfrog: damping sign on u^{n-1}", C,
     "- (1.0 - s) * u_prev[i]", "- (1.0 + s) * u_prev[i]"),
    ("leapfrog: damping sign in the divisor", C,
     "u_next[i] = rhs / (1.0 + s);", "u_next[i] = rhs / (1.0 - s);"),
    ("leapfrog: source subtracted", C,
     "(lap[i] + src)", "(lap[i] - src)"),
    ("forward: source not divided by the cell volume", C,
     "wavelet[(long)t * nsrc + s] * src_w[s * nc + k] / cell;",
     "wavelet[(long)t * nsrc + s] * src_w[s * nc + k];"),
    ("forward: receivers sample u^n instead of u^{n+1}", C,
     "v += rec_w[rr * nc + k] * u_next[rec_idx[rr * nc + k]];",
     "v += rec_w[rr * nc + k] * a[rec_idx[rr * nc + k]];"),
    ("forward: u^{n-1} not rotated", C,
     "        memcpy(b, a, sizeof(double) * tot);\n", "\n"),
    ("adjoint: residual in forward time order", C,
     "residual[(long)(k - 1) * nrec + rr]", "residual[(long)(nt - k) * nrec + rr]"),
    ("adjoint: output scaled by dt instead of dt^2", C,
     "= dt * dt / cell * v;", "= dt / cell * v;"),
    ("imaging: damping term dropped", C,
     "((up - 2.0 * u0 + um) + s * (up - um))", "((up - 2.0 * u0 + um))"),
    ("imaging: second difference with a wrong sign", C,
     "(up - 2.0 * u0 + um)", "(up - 2.0 * u0 - um)"),
    ("layer velocity by reflection instead of replication", PY,
     'np.pad(v, g.nbl, mode="edge")', 'np.pad(v, g.nbl, mode="reflect")'),
    ("sigma_max with log10", PY,
     "math.log(1000.0)", "math.log10(1000.0)"),
    ("linear damping profile", PY,
     "prof = sigma_max * (d / g.nbl) ** 2", "prof = sigma_max * (d / g.nbl)"),
    ("multilinear weights of the two corners swapped", PY,
     "wt *= fr[a] if b else (1.0 - fr[a])", "wt *= (1.0 - fr[a]) if b else fr[a]"),
    ("sparse index without the layer offset", PY,
     "flat += (ks[a] + b + g.nbl) * strides[a]", "flat += (ks[a] + b) * strides[a]"),
    ("centre weight -sum instead of -2 sum", PY,
     "c[0] = -2 * sum(c[1:])", "c[0] = -sum(c[1:])"),
    ("weights with alternating sign flipped", PY,
     "c[j] = Fraction(2 * (-1) ** (j + 1) *", "c[j] = Fraction(2 * (-1) ** j *"),
    ("sinc node window shifted by one", PY,
     "k0 = int(math.floor(t)) - r + 1", "k0 = int(math.floor(t)) - r + 2"),
    ("sinc without its Kaiser window", PY,
     "w.append(sinc * win)", "w.append(sinc * (1.0 if q >= 0.0 else 0.0))"),
    ("sinc nodes without the layer offset", PY,
     "ip = k0 + offs[a] + g.nbl", "ip = k0 + offs[a]"),
    ("sinc nodes outside the grid kept", PY,
     "            if inside:\n                idx[p_i, ci] = flat\n                w[p_i, ci] = wt",
     "            if True:\n                idx[p_i, ci] = flat if inside else 0\n                w[p_i, ci] = wt"),
    ("diffusion step without nu", PY,
     "u = u + nu * dt * laplacian(g, u)", "u = u + dt * laplacian(g, u)"),
    ("diffusion stability limit without the factor 2", PY,
     "return 2.0 / (nu * 4.0 * s_odd", "return 1.0 / (nu * 4.0 * s_odd"),
]


def _tree(tmp, mutant=None):
    """A copy of oracle/, synth/ and the pin tests under tmp, with one
    replacement applied to the oracle copy."""
    os.makedirs(os.path.join(tmp, "oracle"))
    for f in (C, PY):
        shutil.copy(os.path.join(ROOT, "oracle", f), os.path.join(tmp, "oracle", f))
    shutil.copytree(os.path.join(ROOT, "synth"), os.path.join(tmp, "synth"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(tmp, "tests"))
    for f in ("conftest.py", "test_oracle_pins.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(tmp, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(tmp, "tests", "golden"))
    if mutant:
        _, target, old, new = mutant
        path = os.path.join(tmp, "oracle", target)
        src = open(path).read()
        assert src.count(old) == 1, "mutation site not unique: %r" % old
        with open(path, "w") as f:
            f.write(src.replace(old, new))


def _pins(tmp):
    """Run the pins of the tree at tmp in a fresh interpreter; returns the
    pytest exit code (0 all passed, 1 some failed) and the tail of its output."""
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    env.pop("PYTHONPATH", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_oracle_pins.py")],
                       cwd=tmp, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


def test_unmutated_copy_passes(tmp_path):
    _tree(str(tmp_path))
    rc, out = _pins(str(tmp_path))
    assert rc == 0, out


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_a_planted_mistake(mutant, tmp_path):
    _tree(str(tmp_path), mutant)
    rc, out = _pins(str(tmp_path))
    print(mutant[0], "-> pytest exit", rc, "|", out.strip().splitlines()[-1] if out.strip() else "")
    # 1: at least one pin failed (2 or more would be a crash or a collection error)
    assert rc == 1, out
