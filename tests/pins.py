"""Pins for the FP64 oracle: checks against facts the paper and mathematics fix,
never against the oracle itself.  Each pin is a function of the loaded oracle
library so that the mutation test can run the same pins on deliberately broken
builds of the oracle.

Kinds of pins (see each docstring for the passage it rests on):
  * exact rational iterates, worked by hand (tests/golden) and by brute force
    on tiny systems with Python fractions;
  * the solution of A x = b from LAPACK (numpy.linalg.solve);
  * a closed-form family whose iterates and stopping sweep are known exactly;
  * invariants: the fixed point, the contraction bound, power-of-two row
    scaling, column independence, resuming from (x^k, k);
  * special cases: diagonal A, n = 1, integer-exact fixed point, zero
    diagonal, non-finite input, cap L = 0, tol = 0, divergence.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U64 = np.finfo(np.float64).eps / 2  # unit roundoff of binary64


def read_golden(name):
    """Parse a hand-worked fixture: matrix rows separated by '/', rhs, limit,
    then one line per sweep with exact rational entries."""
    A = b = lim = None
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, _, rest = line.partition(" ")
            if tag == "matrix":
                A = [[Fraction(v) for v in r.split()] for r in rest.split("/")]
            elif tag == "rhs":
                b = [Fraction(v) for v in rest.split()]
            elif tag == "limit":
                lim = [Fraction(v) for v in rest.split()]
            else:
                rows.append((int(tag), [Fraction(v) for v in rest.split()]))
    return A, b, lim, rows


def exact_jacobi(A, b, x0, sweeps):
    """Brute-force exact rational Jacobi (component equation of sec. 2).
    Returns the list of iterates x^1..x^sweeps and their max-norm distances."""
    n = len(A)
    x = list(x0)
    its, ds = [], []
    for _ in range(sweeps):
        xn = []
        for i in range(n):
            acc = Fraction(0)
            for j in range(n):
                if j != i:
                    acc += A[i][j] * x[j]
            xn.append((b[i] - acc) / A[i][i])
        ds.append(max(abs(xn[i] - x[i]) for i in range(n)))
        its.append(xn)
        x = xn
    return its, ds


def _f(mat):
    return np.array([[float(v) for v in r] for r in mat], dtype=np.float64)


def pin_hand_2x2(lib):
    """Sec. 2 component equation worked by hand on a 2x2 system (golden)."""
    A, b, lim, rows = read_golden("hand_2x2.txt")
    Af, bf = _f(A), np.array([float(v) for v in b])
    for k, vals in rows:
        x, info = oracle.jacobi(Af, bf, tol=0.0, max_iter=k, lib=lib)
        assert info["status"] == oracle.NOT_CONVERGED and info["iterations"] == k
        want = np.array([float(v) for v in vals[:2]])
        assert np.allclose(x, want, rtol=4 * U64, atol=0), (k, x, want)
        # the distance subtracts two rounded iterates: error within a few ulps of |x|
        assert abs(info["final_delta"] - float(vals[2])) <= 8 * U64 * np.abs(want).max()
    x, info = oracle.jacobi(Af, bf, tol=1e-14, max_iter=200, lib=lib)
    assert info["status"] == oracle.OK
    assert np.allclose(x, [float(v) for v in lim], rtol=1e-13, atol=0)


def pin_hand_3x3(lib):
    """Sec. 2 component equation worked by hand on a 3x3 system (golden)."""
    A, b, lim, rows = read_golden("hand_3x3.txt")
    Af, bf = _f(A), np.array([float(v) for v in b])
    for k, vals in rows:
        x, info = oracle.jacobi(Af, bf, tol=0.0, max_iter=k, lib=lib)
        assert np.allclose(x, [float(v) for v in vals], rtol=4 * U64, atol=0), (k, x)
    x, info = oracle.jacobi(Af, bf, tol=1e-10, max_iter=1000, lib=lib)
    # Exact rational sweeps decide the count: first k with Delta_k < 1e-10.
    _, ds = exact_jacobi(A, b, [Fraction(0)] * 3, 40)
    k_exact = next(i + 1 for i, d in enumerate(ds) if d < Fraction(1, 10**10))
    assert info["status"] == oracle.OK and info["iterations"] == k_exact, (info, k_exact)
    assert np.allclose(x, [1.0, 2.0, 3.0], rtol=0, atol=1e-9)


def pin_brute_force_tiny(lib):
    """Exact rational Jacobi on random tiny dominant systems (n <= 4): every
    iterate within a few ulps, and the same stopping sweep whenever the exact
    distance is not within 1e-6 relative of tol (no tie)."""
    rng = np.random.default_rng(1234)
    for trial in range(12):
        n = 1 + trial % 4
        A = rng.integers(-9, 10, size=(n, n)).astype(np.int64)
        for i in range(n):
            A[i, i] = np.abs(A[i]).sum() - abs(A[i, i]) + rng.integers(1, 5)
            if rng.random() < 0.5:
                A[i, i] = -A[i, i]
        b = rng.integers(-9, 10, size=n)
        x0 = rng.integers(-3, 4, size=n)
        Af = [[Fraction(int(v)) for v in r] for r in A]
        bF = [Fraction(int(v)) for v in b]
        its, ds = exact_jacobi(Af, bF, [Fraction(int(v)) for v in x0], 30)
        for k in (1, 2, 5, 11):
            x, _ = oracle.jacobi(A.astype(float), b.astype(float), X0=x0.astype(float),
                                 tol=0.0, max_iter=k, lib=lib)
            ex = np.array([float(v) for v in its[k - 1]])
            scale = max(1.0, np.abs(ex).max())
            assert np.abs(x - ex).max() <= 16 * k * U64 * scale, (trial, k, x, ex)
        tol = 1e-6
        k_exact = next((i + 1 for i, d in enumerate(ds) if d < Fraction(tol)), None)
        if k_exact is None:
            continue
        margin = min(abs(float(d) - tol) / tol for d in ds[max(0, k_exact - 2):k_exact])
        x, info = oracle.jacobi(A.astype(float), b.astype(float), X0=x0.astype(float),
                                tol=tol, max_iter=30, lib=lib)
        if margin > 1e-6:
            assert info["iterations"] == k_exact and info["status"] == oracle.OK


def pin_lapack_solution(lib):
    """At a tight tolerance the iteration reaches the solution of A x = b that
    LAPACK's LU solve gives (sec. 2: the limit is the solution X)."""
    for n, seed in ((7, 1), (33, 2), (64, 3)):
        A, Xt, B = synth.dominant(n, 3, seed)
        x, info = oracle.jacobi(A, B, tol=1e-15, max_iter=500, lib=lib)
        ref = np.linalg.solve(A, B)
        err = np.abs(x - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, (n, err, info)


def pin_fixed_point_and_contraction(lib):
    """At convergence x = D^-1 (b - (A - D) x) up to ||T||_inf * Delta + O(u);
    and ||x_k - x*||_inf <= ||T|| / (1 - ||T||) * Delta_k (contraction)."""
    A, Xt, B = synth.dominant(96, 1, 77)
    b = B[:, 0]
    d = np.diag(A)
    T = -(A - np.diag(d)) / d[:, None]
    tn = np.abs(T).sum(axis=1).max()
    assert tn < 1.0
    xstar = np.linalg.solve(A, b)
    for tol in (1e-4, 1e-8, 1e-12):
        x, info = oracle.jacobi(A, b, tol=tol, max_iter=1000, lib=lib)
        assert info["status"] == oracle.OK
        delta = info["final_delta"]
        fp = (b - (A @ x - d * x)) / d
        assert np.abs(x - fp).max() <= tn * delta + 64 * U64 * np.abs(x).max()
        bound = tn / (1 - tn) * delta + 64 * U64 * np.abs(xstar).max()
        assert np.abs(x - xstar).max() <= bound


def closed_form(n, a, c, beta, tol):
    """A = a I + c (J - I), b = beta 1, x^0 = 0: x^k = s_k 1 with
    s_k = (beta/a) (1 - r^k) / (1 - r), r = -c (n-1) / a, and
    Delta_k = |beta/a| |r|^(k-1).  Returns (k_stop, s_k_stop, margin), exact."""
    a, c, beta = Fraction(a), Fraction(c), Fraction(beta)
    r = -c * (n - 1) / a
    tolF = Fraction(tol)
    k = 1
    while abs(beta / a) * abs(r) ** (k - 1) >= tolF:
        k += 1
    s = (beta / a) * (1 - r ** k) / (1 - r)
    dk = abs(beta / a) * abs(r) ** (k - 1)
    dprev = abs(beta / a) * abs(r) ** (k - 2) if k > 1 else None
    margins = [abs(float(dk) - tol) / tol]
    if dprev is not None:
        margins.append(abs(float(dprev) - tol) / tol)
    return k, s, min(margins)


def pin_closed_form_family(lib):
    """Constant off-diagonal family: exact iterates and stopping sweep."""
    for n, a, c, beta, tol in ((50, 120, 1, 3, 1e-9), (200, 500, -1, 2, 1e-11),
                               (9, 10, Fraction(1, 2), -1, 1e-7)):
        A = np.full((n, n), float(c))
        np.fill_diagonal(A, float(a))
        b = np.full(n, float(beta))
        k, s, margin = closed_form(n, a, c, beta, tol)
        assert margin > 1e-6
        x, info = oracle.jacobi(A, b, tol=tol, max_iter=1000, lib=lib)
        assert info["status"] == oracle.OK and info["iterations"] == k, (info, k)
        assert np.abs(x - float(s)).max() <= 1e-13 * abs(float(s))


def pin_special_cases(lib):
    """Diagonal A: x^1 = D^-1 b, Delta_2 = 0, stop at sweep 2 (1 when b = 0);
    n = 1; integer-exact fixed point (Delta_1 = 0 exactly, x = X0 bitwise)."""
    d = np.array([2.0, -4.0, 0.5, 8.0])
    A = np.diag(d)
    b = np.array([1.0, 2.0, 3.0, -4.0])
    x, info = oracle.jacobi(A, b, tol=1e-12, max_iter=50, lib=lib)
    assert info["iterations"] == 2 and info["status"] == oracle.OK
    assert np.array_equal(x, b / d)
    x, info = oracle.jacobi(A, np.zeros(4), tol=1e-12, max_iter=50, lib=lib)
    assert info["iterations"] == 1 and np.array_equal(x, np.zeros(4))
    x, info = oracle.jacobi(np.array([[3.0]]), np.array([7.0]), tol=1e-300, max_iter=9, lib=lib)
    assert info["iterations"] == 2 and x[0] == 7.0 / 3.0
    rng = np.random.default_rng(5)
    n = 40
    A = rng.integers(-1, 2, size=(n, n)).astype(np.float64)
    np.fill_diagonal(A, 0.0)
    np.fill_diagonal(A, np.abs(A).sum(axis=1) + 1.0)
    xt = rng.integers(-4, 5, size=(n, 2)).astype(np.float64)
    B = A @ xt
    x, info = oracle.jacobi(A, B, X0=xt, tol=1e-12, max_iter=10, lib=lib)
    assert info["iterations"] == 1 and info["final_delta"] == 0.0
    assert np.array_equal(x, xt)


def pin_tol_zero_and_cap(lib):
    """tol = 0 runs exactly L sweeps even when Delta reaches 0 (strict '<');
    L = 0 returns X^0 with NOT_CONVERGED after 0 sweeps (while k <= L)."""
    A = np.diag([2.0, 4.0])
    b = np.array([1.0, 1.0])
    x, info = oracle.jacobi(A, b, tol=0.0, max_iter=7, lib=lib)
    assert info["iterations"] == 7 and info["status"] == oracle.NOT_CONVERGED
    assert info["final_delta"] == 0.0 and np.array_equal(x, [0.5, 0.25])
    x0 = np.array([9.0, -9.0])
    x, info = oracle.jacobi(A, b, X0=x0, tol=1.0, max_iter=0, lib=lib)
    assert info["iterations"] == 0 and info["status"] == oracle.NOT_CONVERGED
    assert np.array_equal(x, x0)
    A, _, B = synth.dominant(20, 1, 3)
    x5, info = oracle.jacobi(A, B, tol=0.0, max_iter=5, lib=lib)
    x4, _ = oracle.jacobi(A, B, tol=0.0, max_iter=4, lib=lib)
    assert info["status"] == oracle.NOT_CONVERGED and info["iterations"] == 5
    assert info["final_delta"] == np.abs(x5 - x4).max()


def pin_scaling_invariance(lib):
    """Scaling row i and b_i by 2^e_i changes no rounding: every iterate, the
    count and the distance are bitwise unchanged (component equation)."""
    A, _, B = synth.dominant(64, 2, 11)
    e = np.random.default_rng(2).integers(-20, 21, size=64)
    s = np.ldexp(1.0, e)
    x1, i1 = oracle.jacobi(A, B, tol=1e-9, max_iter=100, lib=lib)
    x2, i2 = oracle.jacobi(A * s[:, None], B * s[:, None], tol=1e-9, max_iter=100, lib=lib)
    assert np.array_equal(x1, x2) and i1 == i2


def pin_column_independence(lib):
    """A block of k right-hand sides equals each column solved alone with
    tol = 0 and the block's sweep count (columns never interact)."""
    A, _, B = synth.dominant(48, 5, 21)
    X, info = oracle.jacobi(A, B, tol=1e-10, max_iter=200, lib=lib)
    K = info["iterations"]
    for c in range(5):
        xc, ic = oracle.jacobi(A, B[:, c], tol=0.0, max_iter=K, lib=lib)
        assert np.array_equal(xc, X[:, c])


def pin_resume(lib):
    """The state is only (x^k, k) (step (d) of the pseudocode): resuming from
    x^k with cap L - k equals the uninterrupted run, bitwise."""
    A, _, B = synth.dominant(30, 2, 31)
    full, fi = oracle.jacobi(A, B, tol=0.0, max_iter=12, lib=lib)
    part, _ = oracle.jacobi(A, B, tol=0.0, max_iter=5, lib=lib)
    rest, ri = oracle.jacobi(A, B, X0=part, tol=0.0, max_iter=7, lib=lib)
    assert np.array_equal(full, rest) and ri["final_delta"] == fi["final_delta"]


def pin_failures(lib):
    """alpha_ii = 0 fails (sec. 2), first bad row reported; non-finite
    diagonal, B or X0 rejected; invalid arguments rejected; the paper's own
    U[0,1] inputs (sec. 4) have spectral radius > 1 and diverge."""
    A, _, B = synth.dominant(10, 1, 41)
    Z = A.copy(); Z[3, 3] = 0.0; Z[7, 7] = 0.0
    _, info = oracle.jacobi(Z, B, lib=lib)
    assert info["status"] == oracle.ERR_ZERO_DIAGONAL and info["bad_index"] == 3
    Z = A.copy(); Z[5, 5] = np.nan
    _, info = oracle.jacobi(Z, B, lib=lib)
    assert info["status"] == oracle.ERR_NONFINITE_INPUT and info["bad_index"] == 5
    Bn = B.copy(); Bn[6, 0] = np.inf
    _, info = oracle.jacobi(A, Bn, lib=lib)
    assert info["status"] == oracle.ERR_NONFINITE_INPUT and info["bad_index"] == 6
    x0 = np.zeros(10); x0[2] = np.nan
    _, info = oracle.jacobi(A, B, X0=x0, lib=lib)
    assert info["status"] == oracle.ERR_NONFINITE_INPUT and info["bad_index"] == 2
    for tol, L in ((-1.0, 10), (np.nan, 10), (1e-8, -1)):
        _, info = oracle.jacobi(A, B, tol=tol, max_iter=L, lib=lib)
        assert info["status"] == oracle.ERR_INVALID_ARG
    Ap, bp, x0p = synth.paper_uniform(64, 4)
    d = np.diag(Ap)
    T = -(Ap - np.diag(d)) / d[:, None]
    assert np.abs(np.linalg.eigvals(T)).max() > 1.0
    x, info = oracle.jacobi(Ap, bp, X0=x0p, tol=1e-8, max_iter=10000, lib=lib)
    assert info["status"] == oracle.DIVERGED
    assert not np.isfinite(info["final_delta"]) and 10 < info["iterations"] < 10000


def pin_norms(lib):
    """Max-norm vs the Euclidean distance of sec. 3.1: ||v||_inf <= ||v||_2
    <= sqrt(n k) ||v||_inf, so the L2 rule never stops earlier."""
    A, _, B = synth.dominant(64, 2, 51)
    xi, ii = oracle.jacobi(A, B, tol=0.0, max_iter=6, norm="inf", lib=lib)
    x2, i2 = oracle.jacobi(A, B, tol=0.0, max_iter=6, norm="l2", lib=lib)
    x5, _ = oracle.jacobi(A, B, tol=0.0, max_iter=5, lib=lib)
    v = (xi - x5).ravel()
    assert np.array_equal(xi, x2)
    assert ii["final_delta"] == np.abs(v).max()
    assert abs(i2["final_delta"] - np.linalg.norm(v)) <= 1e-14 * np.linalg.norm(v)
    _, a = oracle.jacobi(A, B, tol=1e-9, max_iter=100, norm="inf", lib=lib)
    _, b = oracle.jacobi(A, B, tol=1e-9, max_iter=100, norm="l2", lib=lib)
    assert b["iterations"] >= a["iterations"]


def pin_planted_solution(lib):
    """b = A X_true makes X_true the solution; the dominant workload of the
    n = 512 FP64 configuration converges to it."""
    A, Xt, B = synth.c1()
    x, info = oracle.jacobi(A, B, tol=1e-10, max_iter=1000, lib=lib)
    assert info["status"] == oracle.OK
    assert np.abs(x - Xt).max() / np.abs(Xt).max() <= 1e-10


def pin_update_and_residual(lib):
    """Single-row updates and the residual agree with dense LAPACK-free numpy
    forms D^-1 (b - (A - D) x) and b - A x to rounding."""
    A, _, B = synth.dominant(70, 3, 61)
    X = np.random.default_rng(3).uniform(-1, 1, size=(70, 3))
    rows = np.array([0, 5, 69, 33])
    d = np.diag(A)
    want = (B - (A @ X - d[:, None] * X)) / d[:, None]
    got = oracle.update_rows(A, B, X, rows, lib=lib)
    assert np.allclose(got, want[rows], rtol=1e-13, atol=1e-15)
    got32 = oracle.update_rows(A.astype(np.float32), B, X, rows, lib=lib)
    A32 = A.astype(np.float32).astype(np.float64)
    d32 = np.diag(A32)
    want32 = (B - (A32 @ X - d32[:, None] * X)) / d32[:, None]
    assert np.allclose(got32, want32[rows], rtol=1e-13, atol=1e-15)
    R = oracle.residual(A, B, X, lib=lib)
    assert np.allclose(R, B - A @ X, rtol=1e-12, atol=1e-12)


def _int_system(rng, n, k, diag_extra=True):
    """Integer matrix (entries -9..9, non-symmetric, a_ii = rowsum + 1..4) and
    integer right-hand sides: every product and partial sum the residual or a
    single update forms is an integer far below 2^53, hence exact in binary64
    in any order."""
    A = rng.integers(-9, 10, size=(n, n)).astype(np.int64)
    np.fill_diagonal(A, 0)
    if diag_extra:
        np.fill_diagonal(A, np.abs(A).sum(axis=1) + rng.integers(1, 5, size=n))
    return A


def pin_residual_exact(lib):
    """R = B - A X (the residual the refinement tests against; the plain
    definition).  Pinned without the oracle's own formula: (1) on a planted
    integer system B = A X_true (formed in int64) R is exactly zero; (2) at
    X_true + E with integer E, R = -A E exactly (int64 product: a transposed
    A, a dropped diagonal term or a sign error changes it); (3) at the
    hand-worked 3x3 iterates (dyadic rationals) R equals the exact rational
    residual bitwise."""
    rng = np.random.default_rng(71)
    for n, k in ((1, 1), (6, 3), (29, 2), (64, 5)):
        A = _int_system(rng, n, k)
        Xt = rng.integers(-4, 5, size=(n, k)).astype(np.int64)
        B = A @ Xt
        R = oracle.residual(A.astype(float), B.astype(float), Xt.astype(float), lib=lib)
        assert np.array_equal(R, np.zeros((n, k))), (n, k)
        E = rng.integers(-3, 4, size=(n, k)).astype(np.int64)
        R = oracle.residual(A.astype(float), B.astype(float), (Xt + E).astype(float), lib=lib)
        assert np.array_equal(R, (-(A @ E)).astype(float)), (n, k)
    Af, b, _, rows = read_golden("hand_3x3.txt")
    for _, vals in rows:
        want = [b[i] - sum(Af[i][j] * vals[j] for j in range(3)) for i in range(3)]
        R = oracle.residual(_f(Af), np.array([float(v) for v in b]),
                            np.array([float(v) for v in vals]), lib=lib)
        assert [Fraction(v) for v in R] == want, (R, want)


def pin_update_rows_exact(lib):
    """One component update at chosen rows (component equation of sec. 2),
    for A in binary64 and in binary32 (the promoted FP32 system).  On integer
    inputs the sum is exact, so the result is the correctly rounded quotient
    (b_i - sum_{j != i} a_ij x_j) / a_ii, which Python's integer true division
    gives exactly; and on random inputs it equals bitwise the row of one sweep
    of the pinned driver (tol = 0, L = 1) started from the same iterate."""
    rng = np.random.default_rng(72)
    for n, k in ((1, 1), (5, 2), (40, 3)):
        A = _int_system(rng, n, k)
        B = rng.integers(-50, 51, size=(n, k)).astype(np.int64)
        X = rng.integers(-7, 8, size=(n, k)).astype(np.int64)
        rows = np.unique(rng.integers(0, n, size=min(n, 6)))
        want = np.empty((rows.size, k))
        for r, i in enumerate(rows):
            for c in range(k):
                s = sum(int(A[i, j]) * int(X[j, c]) for j in range(n) if j != i)
                want[r, c] = (int(B[i, c]) - s) / int(A[i, i])
        for Aform in (A.astype(np.float64), A.astype(np.float32)):
            got = oracle.update_rows(Aform, B.astype(float), X.astype(float), rows, lib=lib)
            assert np.array_equal(got, want), (n, k, Aform.dtype)
    for n, k in ((17, 1), (96, 4)):
        A32, _, B32 = synth.dominant_f32(n, k, 900 + n)
        A64, B64 = A32.astype(np.float64), B32.astype(np.float64)
        X0 = rng.uniform(-1, 1, size=(n, k))
        x1, info = oracle.jacobi(A64, B64, X0=X0, tol=0.0, max_iter=1, lib=lib)
        assert info["iterations"] == 1
        rows = np.arange(n)
        for Aform in (A64, A32):
            got = oracle.update_rows(Aform, B64, X0, rows, lib=lib)
            assert np.array_equal(got, x1.reshape(n, k)), (n, k, Aform.dtype)


PINS = [pin_hand_2x2, pin_hand_3x3, pin_brute_force_tiny, pin_lapack_solution,
        pin_fixed_point_and_contraction, pin_closed_form_family, pin_special_cases,
        pin_tol_zero_and_cap, pin_scaling_invariance, pin_column_independence, pin_resume,
        pin_failures, pin_norms, pin_planted_solution, pin_update_and_residual,
        pin_residual_exact, pin_update_rows_exact]
