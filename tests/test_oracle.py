"""The oracle checked against its pins (CPU only), plus a mutation test that
plants plausible mistakes in copies of the oracle source and requires every
mutant to fail at least one pin."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
import pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("pin", pins.PINS, ids=[p.__name__ for p in pins.PINS])
def test_pin(pin):
    pin(oracle.load())


def test_tie_case_is_detected():
    """2x2 at tol 1e-10: exact arithmetic gives Delta_20 = 1e-10 exactly (stop
    at 21) while FP64 rounds it just below (stop at 20).  The tie margin rule
    flags it, so no count parity is claimed there."""
    from fractions import Fraction
    A = [[Fraction(4), Fraction(1)], [Fraction(2), Fraction(5)]]
    b = [Fraction(1), Fraction(2)]
    _, ds = pins.exact_jacobi(A, b, [Fraction(0)] * 2, 25)
    assert ds[19] == Fraction(1, 10**10)
    x, info = oracle.jacobi(np.array([[4.0, 1], [2, 5]]), np.array([1.0, 2]), tol=1e-10,
                            max_iter=100)
    assert info["iterations"] == 20
    assert abs(float(ds[19]) - 1e-10) / 1e-10 < 1e-6  # inside the tie margin
    x, info = oracle.jacobi(np.array([[4.0, 1], [2, 5]]), np.array([1.0, 2]), tol=2e-10,
                            max_iter=100)
    k_exact = next(i + 1 for i, d in enumerate(ds) if d < Fraction(2, 10**10))
    assert info["iterations"] == k_exact == 20


def test_round_bf16_against_library_and_special_values():
    """RNE to bfloat16: float32 inputs (no double rounding possible) agree with
    torch's conversion; boundary values follow IEEE round-to-nearest-even."""
    import torch
    rng = np.random.default_rng(0)
    f = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.uniform(-1, 1, 5000)]).astype(np.float32)
    want = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.round_bf16(f.astype(np.float64))
    assert np.array_equal(got, want)
    r = oracle.round_bf16
    assert r([1.0 + 2.0**-8])[0] == 1.0                      # tie -> even (down)
    assert r([1.0 + 3 * 2.0**-8])[0] == 1.0 + 2.0**-6        # tie -> even (up)
    assert r([1.0 + 2.0**-8 + 2.0**-40])[0] == 1.0 + 2.0**-7  # above tie: up
    assert r([np.ldexp(255.0, 120)])[0] == np.ldexp(255.0, 120)
    assert np.isinf(r([np.ldexp(255.5, 120)])[0])
    assert r([2.0**-133])[0] == 2.0**-133                     # smallest subnormal
    assert r([2.0**-134])[0] == 0.0                           # tie to even zero
    assert r([-0.0])[0] == 0.0 and np.isnan(r([np.nan])[0])


# Mutants: (description, original text, replacement).  Each is a plausible
# mistake in transcribing the paper's method.
MUTANTS = [
    ("b dropped", "return (B[i * ldb + c] - s) / row[i];", "return (0.0 - s) / row[i];"),
    ("b sign", "return (B[i * ldb + c] - s) / row[i];", "return (-B[i * ldb + c] - s) / row[i];"),
    ("sum sign", "        s = s + p;\n    }\n    (void)k;", "        s = s - p;\n    }\n    (void)k;"),
    ("transposed A", "double p = row[j] * Xold[j * ldo + c];",
     "double p = A[j * lda + i] * Xold[j * ldo + c];"),
    ("diagonal kept", "        if (j == i) continue;\n        double p = row[j]",
     "        double p = row[j]"),
    ("pseudocode garble (b inside sum)", "double p = row[j] * Xold[j * ldo + c];",
     "double p = row[j] * Xold[j * ldo + c] - B[i * ldb + c];"),
    ("old iterate returned", "if (delta < tol) { status = ORACLE_OK; result = Xn; break; }",
     "if (delta < tol) { status = ORACLE_OK; result = Xt; break; }"),
    ("non-strict test", "if (delta < tol) {", "if (delta <= tol) {"),
    ("count off by one", "iters = it;", "iters = it + 1;"),
    ("in-place update (Gauss-Seidel)",
     "Xn[i * k + c] = oracle_component(n, k, A, lda, B, ldb, Xt, k, i, c);",
     "Xt[i * k + c] = Xn[i * k + c] = oracle_component(n, k, A, lda, B, ldb, Xt, k, i, c);"),
    ("max-norm replaced by first entry", "} else if (d > acc) {", "} else if (t == 0) {"),
    ("zero diagonal unchecked", "if (d == 0.0) { *bad = i; return ORACLE_ERR_ZERO_DIAGONAL; }",
     ""),
    ("l2 without sqrt", "return norm == ORACLE_NORM_L2 ? sqrt(acc) : acc;", "return acc;"),
    # the residual R = B - A X used by the refinement checks
    ("residual sign", "R[i * ldr + c] = B[i * ldb + c] - s;", "R[i * ldr + c] = s - B[i * ldb + c];"),
    ("residual drops the diagonal term",
     "                double p = A[i * lda + j] * X[j * ldx + c];",
     "                if (j == i) continue;\n                double p = A[i * lda + j] * X[j * ldx + c];"),
    ("residual transposed A", "double p = A[i * lda + j] * X[j * ldx + c];",
     "double p = A[j * lda + i] * X[j * ldx + c];"),
    ("residual reads column 0 only", "double p = A[i * lda + j] * X[j * ldx + c];",
     "double p = A[i * lda + j] * X[j * ldx];"),
    # single-row updates (binary64 and the promoted binary32 matrix)
    ("row update of the wrong row",
     "oracle_component(n, k, A, lda, B, ldb, Xold, ldo, rows[r], c);",
     "oracle_component(n, k, A, lda, B, ldb, Xold, ldo, r, c);"),
    ("f32 row update keeps the diagonal",
     "                if (j == i) continue;\n                double p = (double)row[j]",
     "                double p = (double)row[j]"),
    ("f32 row update b sign", "out[r * k + c] = (B[i * ldb + c] - s) / (double)row[i];",
     "out[r * k + c] = (-B[i * ldb + c] - s) / (double)row[i];"),
    ("f32 row update transposed A", "double p = (double)row[j] * Xold[j * ldo + c];",
     "double p = (double)A[j * lda + i] * Xold[j * ldo + c];"),
]


@pytest.mark.parametrize("desc,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, desc, old, new):
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, desc
    mutated = src.replace(old, new, 1)
    cpath = tmp_path / "mutant.c"
    cpath.write_text(mutated)
    so = str(tmp_path / "libmutant.so")
    oracle.build(src=str(cpath), out=so)
    lib = oracle.load(so)
    failed = []
    for pin in pins.PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"mutant '{desc}' passed every pin"
