"""The oracle's pins catch plausible mistakes: each case plants one mistake in a copy of
oracle/hawkes_oracle.c (on the CPU, in a temporary directory), builds it, and checks that at
least one pin of tests/test_oracle_pins.py fails against it."""

import importlib.util
import os
import re
import shutil

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hawkes_oracle.c")

# (description, regex, replacement)
MUTATIONS = [
    ("target bandwidth instead of source", r"const double h = h0 \* s\[m\];", "const double h = h0 * s[nt];"),
    ("dropped -2/tau_x derivative term", r"\(d2 / \(taux \* taux \* taux\) - 2\.0 / taux\)", "(d2 / (taux * taux * taux))"),
    ("ties kept in both sums", r"if \(t\[m\] == tn\)", "if (m == nt)"),
    ("1-D density normalised as 2-D", r"return exp\(-d \* d / \(2\.0 \* v\)\) / sqrt\(2\.0 \* M_PI \* v\);",
     "return exp(-d * d / (2.0 * v)) / (2.0 * M_PI * v);"),
    ("compensator sign", r"out\[0\] = mu \* bg \+ xi \* \(1\.0 - ea\);", "out[0] = mu * bg + xi * (1.0 + ea);"),
    ("missing lower time limit", r" - std_normal_cdf\(-tm / taut\);", ";"),
    ("omega read as a time scale", r"exp\(-omega \* dt\);", "exp(-dt / omega);"),
    ("omega derivative sign", r"\(1\.0 / omega - dt\)", "(1.0 / omega + dt)"),
    ("compensator omega derivative lacks xi", r"out\[1 \+ P_OMEGA\] = xi \* a \* ea;", "out[1 + P_OMEGA] = a * ea;"),
    ("2-D density missing a factor 2", r"return exp\(-r2 / \(2\.0 \* v\)\) / \(2\.0 \* M_PI \* v\);",
     "return exp(-r2 / (2.0 * v)) / (M_PI * v);"),
    ("h0 derivative exponent", r"\(d2 / \(h \* h \* h0\) - 2\.0 / h0\)", "(d2 / (h * h * h0) - 1.0 / h0)"),
    ("transposed coordinate", r"const double dx = xn - x\[m\], dy = yn - y\[m\];",
     "const double dx = xn - x[m], dy = yn - x[m];"),
    ("time horizon past the last event", r"double tN = t\[0\];", "double tN = t[n - 1] + 1.0;"),
    ("no floor", r"const int floored = lam_i < ORACLE_LAMBDA_FLOOR;", "const int floored = 0;"),
    ("tau_t derivative exponent", r"\(dt \* dt / \(taut \* taut \* taut\) - 1\.0 / taut\)",
     "(dt * dt / (taut * taut) - 1.0 / taut)"),
    ("Philox round multiplier", r"0xD2E7470EE14C6C93ULL", "0xD2E7470EE14C6C95ULL"),
    ("x and y from the same uniform", r"const double uy = \(double\)\(w\[1\] >> 11\)",
     "const double uy = (double)(w[0] >> 11)"),
    ("uniform background without 1/A", r"const double beta = n1_density\(dt, taut \* taut\) / area;",
     "const double beta = n1_density(dt, taut * taut);"),
    ("uniform background keeps the spatial Gaussian", r"const double beta = n1_density\(dt, taut \* taut\) / area;",
     "const double beta = n2_density(d2, taux * taux) * n1_density(dt, taut * taut) / area;"),
]

PIN_TESTS = [name for name in dir(pins) if name.startswith("test_")]


def _load_mutant(tmpdir, src_text):
    d = os.path.join(tmpdir, "oracle")
    os.makedirs(d, exist_ok=True)
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), os.path.join(d, "__init__.py"))
    with open(os.path.join(d, "hawkes_oracle.c"), "w") as f:
        f.write(src_text)
    spec = importlib.util.spec_from_file_location("oracle_mutant", os.path.join(d, "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build(force=True)
    return mod


@pytest.mark.parametrize("desc,pattern,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(desc, pattern, repl, tmp_path, monkeypatch):
    src = open(SRC).read()
    mutated, count = re.subn(pattern, repl, src)
    assert count >= 1, f"mutation '{desc}' did not apply"
    mod = _load_mutant(str(tmp_path), mutated)
    monkeypatch.setattr(pins, "oracle", mod)
    failed = []
    for name in PIN_TESTS:
        fn = getattr(pins, name)
        params = getattr(fn, "pytestmark", [])
        if params:  # no parametrised pins in the file; guard against future ones
            continue
        try:
            fn()
        except AssertionError:
            failed.append(name)
        except Exception:  # a crash or invalid result also counts as caught
            failed.append(name)
        if failed:
            break
    assert failed, f"no pin fails for the planted mistake: {desc}"


# ------------------------------------------------------------ the MLP reference

import test_mlp_oracle as mlp_pins  # noqa: E402

MLP_SRC = os.path.join(ROOT, "oracle", "mlp.py")
MLP_MUTATIONS = [
    ("missing GELU curvature term", r"h3_bar = a3_bar \* s3 \+ s3_bar \* gelu_d2\(h3\)", "h3_bar = a3_bar * s3"),
    ("transposed weight in the input gradient", r"d2 = \(d3 @ p\[\"W3\"\]\) \* gelu_d1\(h2\)",
     'd2 = (d3 @ p["W3"].T) * gelu_d1(h2)'),
    ("transposed weight in the loss's reverse pass", r"c2 = d3 @ W3 ", "c2 = d3 @ W3.T "),
    ("W1 gradient without the reverse-pass term", r"grad\[\"W1\"\] = d1\.T @ gz_bar", 'grad["W1"] = 0.0 * gz_bar.T @ d1'),
    ("slope adjoint from the wrong factor", r"s2_bar = d2_bar \* c2", "s2_bar = d2_bar * s2"),
    ("GELU derivative without x phi(x)", r"return 0\.5 \* \(1\.0 \+ _erf\(x / _SQ2\)\) \+ x \* _ISQ2PI \* np\.exp\(-0\.5 \* x \* x\)",
     "return 0.5 * (1.0 + _erf(x / _SQ2))"),
    ("Adam without bias correction", r"mh = m / \(1\.0 - beta1 \*\* step\)", "mh = m"),
    ("Adam first moment decayed by beta2", r"m = beta1 \* m \+", "m = beta2 * m +"),
    ("Adam second moment decayed by beta1", r"v = beta2 \* v \+", "v = beta1 * v +"),
    ("Adam second moment bias-corrected with beta1", r"vh = v / \(1\.0 - beta2 \*\* step\)", "vh = v / (1.0 - beta1 ** step)"),
    ("gradient-matching weight dropped", r"gz_bar = \(2\.0 \* lam / B\) \* r", "gz_bar = 0.0 * r"),
]
MLP_PIN_TESTS = [name for name in dir(mlp_pins) if name.startswith("test_")]


@pytest.mark.parametrize("desc,pattern,repl", MLP_MUTATIONS, ids=[m[0] for m in MLP_MUTATIONS])
def test_mlp_pins_catch_planted_mistake(desc, pattern, repl, tmp_path, monkeypatch):
    src = open(MLP_SRC).read()
    mutated, count = re.subn(pattern, repl, src)
    assert count >= 1, f"mutation '{desc}' did not apply"
    path = os.path.join(str(tmp_path), "mlp_mutant.py")
    with open(path, "w") as f:
        f.write(mutated)
    spec = importlib.util.spec_from_file_location("mlp_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mlp_pins, "mlp", mod)
    failed = []
    for name in MLP_PIN_TESTS:
        try:
            getattr(mlp_pins, name)()
        except Exception:
            failed.append(name)
            break
    assert failed, f"no MLP pin fails for the planted mistake: {desc}"
