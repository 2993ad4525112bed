"""GPU parity of mixed-precision iterative refinement (FP32 / BF16 sweeps,
FP64 residual and update) against the FP64 oracle's tight solution x_ref.

The iteration counts of refinement depend on reduced-precision rounding and
are parity unpinned; the result is compared with x_ref (the plain FP64 oracle
run to 1e-15), and the residual is recomputed by the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_REFINE, dev, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jac(gpu):
    import paper_1403_5805_amd as jac
    return jac


def _xref(A, B):
    x, info = oracle.jacobi(A, B, tol=1e-15, max_iter=1000)
    return x


@pytest.mark.parametrize("lo", ["bf16", "f32"])
@pytest.mark.parametrize("n,k", [(1024, 1), (777, 4), (300, 16)])
def test_refine_parity(jac, lo, n, k):
    A, Xt, B = synth.dominant(n, k, 4000 + n + k, synth.MULTIPLICATIVE, 0.5, 1.0)
    xr = _xref(A, B)
    say("refine", lo, n, k)
    X, info = jac.solve(dev(A), dev(B), mode="refine", sweep_dtype=lo)
    assert info["status"] == jac.OK, info
    assert info["rel_residual"] < 1e-12
    assert info["outer_iterations"] >= 2
    assert rel_err(host(X), xr) <= REL_REFINE
    R = oracle.residual(A, B, host(X))
    assert np.linalg.norm(R) / np.linalg.norm(B) < 1e-10


def _padded(A, pad):
    """Device copy of A with leading dimension n + pad (odd pad: rows not
    16-byte aligned)."""
    import torch
    n = A.shape[0]
    big = torch.zeros((n, n + pad), dtype=torch.float64)
    big[:, :n] = torch.from_numpy(A)
    return big.cuda()[:, :n]


@pytest.mark.parametrize("n,k,pad", [(1, 3, 0), (17, 5, 0), (129, 2, 0), (515, 3, 1),
                                     (1000, 8, 0), (777, 17, 1), (2047, 32, 0)])
def test_refine_multi_rhs_parity(jac, n, k, pad):
    """Several right-hand sides: the FP64 residual runs on MFMA tiles (k >= 2)
    and the inner solve on the FP32 MFMA kernel (k >= 3); odd leading
    dimensions take the unaligned load path; n = 1 and ragged n cover the
    partial tiles and column blocks."""
    mode = synth.ADDITIVE if n < 32 else synth.MULTIPLICATIVE
    lo_m, hi_m = (1.0, 2.0) if n < 32 else (0.5, 1.0)
    A, Xt, B = synth.dominant(n, k, 4200 + n + k, mode, lo_m, hi_m)
    xr = _xref(A, B)
    Ad = _padded(A, pad)
    for lo in ("bf16", "f32"):
        say("refine multi-rhs", lo, n, k, pad)
        X, info = jac.solve(Ad, dev(B), mode="refine", sweep_dtype=lo)
        assert info["status"] == jac.OK, info
        assert info["rel_residual"] < 1e-12
        assert rel_err(host(X), xr) <= REL_REFINE, (lo, n, k)
        R = oracle.residual(A, B, host(X))
        assert np.linalg.norm(R) / np.linalg.norm(B) < 1e-10


@pytest.mark.parametrize("n,k,pad", [(1, 2, 0), (63, 4, 1), (300, 16, 0), (1001, 17, 1),
                                     (4099, 32, 0), (2000, 1, 0)])
def test_fp64_residual_pass(jac, n, k, pad):
    """One residual pass from a random x0 (max_outer = 0): X comes back as x0
    bitwise and ||B - A x0||_2 / ||B||_2 matches the oracle's residual (no
    cancellation, so the two agree to rounding)."""
    A, _, B = synth.dominant(n, k, 4300 + n + k, synth.ADDITIVE, 1.0, 2.0)
    x0 = np.random.default_rng(n + k).uniform(-1, 1, size=(n, k))
    say("fp64 residual", n, k, pad)
    X, info = jac.solve(_padded(A, pad), dev(B), dev(x0), mode="refine", max_outer=0)
    assert info["status"] == jac.NOT_CONVERGED and info["outer_iterations"] == 1
    assert np.array_equal(host(X), x0)
    ref = np.linalg.norm(oracle.residual(A, B, x0)) / np.linalg.norm(B)
    assert abs(info["rel_residual"] - ref) <= 1e-12 * ref


def test_refine_caps_and_x0(jac):
    """max_outer = 0 returns X0 after one residual evaluation; a good X0 is
    accepted at once (one residual pass, no inner sweep)."""
    A, Xt, B = synth.dominant(500, 2, 4100, synth.MULTIPLICATIVE, 0.5, 1.0)
    x0 = np.random.default_rng(0).uniform(-1, 1, size=(500, 2))
    say("refine caps")
    X, info = jac.solve(dev(A), dev(B), dev(x0), mode="refine", max_outer=0)
    assert info["status"] == jac.NOT_CONVERGED and info["outer_iterations"] == 1
    assert np.array_equal(host(X), x0)
    xr = _xref(A, B)
    X, info = jac.solve(dev(A), dev(B), dev(xr), mode="refine")
    assert info["status"] == jac.OK and info["outer_iterations"] == 1
    assert info["iterations"] == 0
    Z = A.copy(); Z[7, 7] = 0.0
    X, info = jac.solve(dev(Z), dev(B), mode="refine")
    assert info["status"] == jac.ERR_ZERO_DIAGONAL and info["bad_index"] == 7


def test_c4_full_size(jac):
    """n = 32768, FP64 A stored BF16 for the sweeps (2 GiB) with the FP64 A
    (8 GiB) kept on the device for the residual.  The configuration's stop
    rule ||r||_2/||b||_2 < 1e-10 leaves a max-norm error of 1.5e-10 on this
    system (measured: the error/residual ratio is about 15), so the default
    residual target is 1e-12; the residual is recomputed by the oracle and x is
    compared with x_ref at the 1e-10 bar."""
    import torch
    A, Xt, B = synth.c4()
    b = B[:, 0]
    say("c4 n=32768")
    Ad = torch.from_numpy(A).cuda()
    X, info = jac.solve(Ad, dev(b), mode="refine", sweep_dtype="bf16")
    assert info["status"] == jac.OK, info
    x = host(X)
    del Ad
    torch.cuda.empty_cache()
    R = oracle.residual(A, b, x)
    assert np.linalg.norm(R) / np.linalg.norm(b) < 1e-10
    xr = _xref(A, b)
    assert rel_err(x, xr) <= REL_REFINE
    print(f"c4: outer={info['outer_iterations']} inner={info['iterations']} "
          f"rel_res={info['rel_residual']:.3e} err_vs_xref={rel_err(x, xr):.3e} "
          f"device_ms={info['device_ms']:.1f}", flush=True)


@pytest.mark.parametrize("lo", ["bf16", "f32"])
@pytest.mark.parametrize("n,pad", [(2, 0), (37, 1), (1024, 0), (1031, 1), (9000, 0)])
def test_fused_conversion_bitwise(jac, monkeypatch, lo, n, pad):
    """From a given x0 with one right-hand side, the first residual pass
    writes A_lo while it streams A: the reduced copy equals the conversion
    kernel's bitwise, so the whole refinement (X, counts, residual) is bitwise
    the same as with a separate conversion pass.  From x0 = 0 the first
    residual is B itself (no pass over A): bitwise the same as passing an
    explicit zero x0.  Odd leading dimensions take the unaligned (element)
    path, n = 9000 several staged x chunks."""
    import torch
    A, _, B = synth.dominant(n, 1, 4100 + n + pad, synth.MULTIPLICATIVE, 0.5, 1.0)
    Ad = _padded(A, pad)
    Bd = dev(B)
    x0 = dev(np.random.default_rng(n).uniform(-1, 1, size=(n, 1)))
    out = {}
    for fused in ("0", "1"):
        monkeypatch.setenv("JACOBI_REFINE_FUSED_CONVERT", fused)
        say("fused conversion", lo, n, pad, fused)
        out[fused] = jac.solve(Ad, Bd, x0, mode="refine", sweep_dtype=lo)
    monkeypatch.delenv("JACOBI_REFINE_FUSED_CONVERT")
    say("zero start", lo, n, pad)
    out["none"] = jac.solve(Ad, Bd, mode="refine", sweep_dtype=lo)
    out["zeros"] = jac.solve(Ad, Bd, torch.zeros_like(Bd), mode="refine", sweep_dtype=lo)
    for a, b in (("0", "1"), ("none", "zeros")):
        (X0, i0), (X1, i1) = out[a], out[b]
        assert i1["status"] == jac.OK, (b, i1)
        for key in ("status", "iterations", "outer_iterations", "rel_residual", "final_delta"):
            assert i0[key] == i1[key], (a, b, key, i0, i1)
        assert torch.equal(X0, X1), (a, b)


@pytest.mark.parametrize("k", [1, 3])
def test_zero_start_edges(jac, k):
    """From x0 = 0 the first residual is B: B = 0 is solved at once by x = 0
    (relative residual 0, no inner sweep); with max_outer = 0 the call
    returns x = 0 with relative residual 1."""
    import torch
    A, _, B = synth.dominant(300, k, 4200 + k, synth.MULTIPLICATIVE, 0.5, 1.0)
    say("zero start edges", k)
    X, info = jac.solve(dev(A), dev(np.zeros_like(B)), mode="refine")
    assert info["status"] == jac.OK and info["outer_iterations"] == 1
    assert info["iterations"] == 0 and info["rel_residual"] == 0.0
    assert not bool(torch.any(X != 0))
    X, info = jac.solve(dev(A), dev(B), mode="refine", max_outer=0)
    assert info["status"] == jac.NOT_CONVERGED and info["outer_iterations"] == 1
    assert info["rel_residual"] == 1.0
    assert not bool(torch.any(X != 0))


def _rounding_system(n, fmt, seed):
    """FP64 system whose entries sit on, just inside and exactly at the
    rounding points of the reduced format (bf16: 8 significant bits, f32: 24),
    built so that two FP32-accumulated sweeps on the correctly rounded copy
    are exact.

    * diagonal: +-2^t (t in 2..4) plus an offset of half a unit above (a tie,
      rounds down to the even 2^t), a quarter unit below (the tie between 2^t
      and the value below, whose spacing is half as wide), or just inside
      either tie; a few rows use a diagonal near 2^-130 (subnormal in both
      formats) with a tie offset and b = 2^-120, so that d = 2^10;
    * b: small integers, so d^(1) = b / 2^t has at most four significant bits;
    * off-diagonals of the rows with b != 0: a few short values (v in
      {0.375, 0.625, 0.75, 0.875, 1.25, 1.5}, either sign) on or inside a tie
      of v, all of which round to v; every product and partial sum of the
      second sweep is then exact in FP32 in any order;
    * rows with b = 0 (d = 0 in both sweeps) only meet columns of other such
      rows; their columns carry values that matter only for the rounding
      itself: long random values, subnormal-range values and values just below
      the overflow threshold (rounded to the largest finite value, never to
      inf, which times d = 0 would give NaN).
    Returns (A, b) with A in FP64."""
    p = 8 if fmt == "bf16" else 24
    rng = np.random.default_rng(seed)
    ulp = lambda v: 2.0 ** (np.floor(np.log2(abs(v))) - (p - 1))  # noqa: E731
    A = np.zeros((n, n))
    b = np.zeros(n)
    kind = rng.choice(3, size=n, p=[0.2, 0.7, 0.1])  # 0: b = 0, 1: ordinary, 2: subnormal diag
    kind[0], kind[1], kind[2] = 0, 1, 2
    zero = np.flatnonzero(kind == 0)
    live = np.flatnonzero(kind == 1)
    inside = 0.5 - 2.0 ** -12
    for i in range(n):
        sgn = rng.choice([-1.0, 1.0])
        if kind[i] == 2:
            v = 2.0 ** -130
            q = 2.0 ** (-133 if fmt == "bf16" else -149)
            A[i, i] = sgn * (v + rng.choice([0.5, -0.5, inside, -inside, 0.0]) * q)
            b[i] = sgn * 2.0 ** -120
            continue
        v = 2.0 ** rng.integers(2, 5)
        u = ulp(v)
        A[i, i] = sgn * (v + rng.choice([0.5, -0.25, inside * 1.0, -inside / 2, 0.0]) * u)
        if kind[i] == 0:
            for j in rng.choice(zero, size=min(4, len(zero)), replace=False):
                if j != i:
                    A[i, j] = rng.uniform(-1, 1)
            continue
        b[i] = rng.choice([-1.0, 1.0]) * rng.integers(1, 9)
        for j in rng.choice(live, size=min(5, len(live)), replace=False):
            if j == i:
                continue
            w = rng.choice([0.375, 0.625, 0.75, 0.875, 1.25, 1.5]) * rng.choice([-1.0, 1.0])
            A[i, j] = w + rng.choice([0.5, -0.5, inside, -inside, 0.25, 0.0]) * ulp(w)
    # columns of b = 0 rows in ordinary rows: values whose rounding does not
    # reach the result
    top = (2.0 - 2.0 ** -(p - 1)) * 2.0 ** 127  # largest finite value of the format
    for i in live:
        for j in rng.choice(zero, size=min(3, len(zero)), replace=False):
            c = rng.integers(3)
            if c == 0:
                A[i, j] = rng.uniform(-1, 1)
            elif c == 1:
                A[i, j] = rng.choice([-1.0, 1.0]) * (2.0 ** -131 + 2.0 ** -135)
            else:
                A[i, j] = rng.choice([-1.0, 1.0]) * (top + 0.25 * 2.0 ** (127 - (p - 1)))
    return A, b


@pytest.mark.parametrize("fmt", ["bf16", "f32"])
@pytest.mark.parametrize("n,k,pad,x0", [(40, 1, 0, None), (203, 1, 1, None), (203, 1, 0, "zero"),
                                        (129, 1, 1, "zero"), (97, 3, 1, None), (150, 8, 0, None),
                                        (75, 16, 1, None)])
def test_reduced_copy_rounding_bitwise(jac, fmt, n, k, pad, x0):
    """The device's reduced copy A_lo = RNE(A) against the oracle's rounding.

    From x = 0, one correction with two inner sweeps (max_outer = 1,
    max_inner = 2) returns X = d^(2), the second Jacobi iterate on
    (A_lo, fl32(B)).  On the system of _rounding_system every step of that
    iterate is exact in FP32 when A_lo is rounded correctly, so X must equal
    the oracle's two sweeps on the oracle-rounded copy bitwise.  Covered:
    the conversion kernel (x0 = None, or k > 1) and the first residual pass
    that writes A_lo while it streams A (an explicit zero x0 with one column),
    aligned and odd leading dimensions, the vector sweep (k < 8) and the MFMA
    sweep (k >= 3)."""
    A, b = _rounding_system(n, fmt, 4500 + n + k + pad)
    B = np.repeat(b[:, None], k, axis=1) * (1.0 + (np.arange(k) % 2))[None, :]
    lo = oracle.round_bf16(A) if fmt == "bf16" else A.astype(np.float32).astype(np.float64)
    assert np.all(np.isfinite(lo))
    xe, io = oracle.jacobi(lo, B.astype(np.float32).astype(np.float64), tol=0.0, max_iter=2)
    assert io["iterations"] == 2
    Bd = dev(B)
    xd = None if x0 is None else dev(np.zeros_like(B))
    say("reduced copy rounding", fmt, n, k, pad, x0)
    X, info = jac.solve(_padded(A, pad), Bd, xd, mode="refine", sweep_dtype=fmt, max_outer=1,
                        max_inner=2)
    assert info["status"] in (jac.OK, jac.NOT_CONVERGED), info
    assert info["iterations"] == 2 and info["outer_iterations"] == 2, info
    x = host(X).reshape(n, k)
    bad = np.flatnonzero((x != np.asarray(xe).reshape(n, k)).any(axis=1))
    assert bad.size == 0, (fmt, bad[:8], x[bad[:4]], np.asarray(xe).reshape(n, k)[bad[:4]])


@pytest.mark.parametrize("lo", ["bf16", "f32"])
@pytest.mark.parametrize("n,k,x0", [(1500, 1, False), (1500, 1, True), (600, 4, False),
                                    (333, 16, True)])
def test_prepared_matrix(jac, lo, n, k, x0):
    """A prepared matrix (jacobi_matrix_create) keeps A and, for refinement, its
    reduced copy built once: every refine solve on it, for several right-hand
    sides, equals jacobi_solve's refine solve of the same system bitwise (the
    same rounding of A, built by the conversion kernel or by the fused first
    residual pass), and so do plain solves; a sweep dtype other than the
    prepared one, or a reduced copy of a non-FP64 matrix, is refused."""
    import torch
    A, Xt, B = synth.dominant(n, k, 4700 + n + k, synth.MULTIPLICATIVE, 0.5, 1.0)
    Ad = dev(A)
    m = jac.Matrix(Ad, sweep_dtype=lo)
    xr = _xref(A, B)
    for rep, scale in enumerate((1.0, -0.5, 2.0)):
        Bd = dev(B * scale)
        X0 = dev(np.random.default_rng(rep).uniform(-1, 1, size=B.shape)) if x0 else None
        say("prepared matrix", lo, n, k, x0, rep)
        Xp, ip = m.solve(Bd, X0, mode="refine", sweep_dtype=lo)
        Xs, is_ = jac.solve(Ad, Bd, X0, mode="refine", sweep_dtype=lo)
        assert ip["status"] == is_["status"] == jac.OK, (ip, is_)
        assert torch.equal(Xp, Xs)
        assert ip["iterations"] == is_["iterations"]
        assert ip["outer_iterations"] == is_["outer_iterations"]
        assert rel_err(host(Xp), xr * scale) <= REL_REFINE
    Xp, ip = m.solve(dev(B), tol=1e-11, max_iter=500)
    Xs, is_ = jac.solve(Ad, dev(B), tol=1e-11, max_iter=500)
    assert ip["status"] == jac.OK and torch.equal(Xp, Xs) and ip["iterations"] == is_["iterations"]
    other = "f32" if lo == "bf16" else "bf16"
    _, bad = m.solve(dev(B), mode="refine", sweep_dtype=other)
    assert bad["status"] == jac.ERR_INVALID_ARG
    m.close()
    with pytest.raises(RuntimeError):
        jac.Matrix(Ad.float(), sweep_dtype=lo)
    m32 = jac.Matrix(Ad.float())  # no reduced copy: plain solves only
    X32, i32 = m32.solve(dev(B.astype(np.float32)), tol=1e-6, max_iter=500)
    Y32, j32 = jac.solve(Ad.float(), dev(B.astype(np.float32)), tol=1e-6, max_iter=500)
    assert torch.equal(X32, Y32) and i32["iterations"] == j32["iterations"]
    m32.close()
