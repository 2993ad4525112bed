"""GPU parity of the plain Jacobi path (jacobi_solve) against the FP64 oracle.

Bars: FP64 sweeps match the oracle's iteration count (when the tie margin
holds) and agree to 1e-12 norm-wise relative; FP32 / BF16-A sweeps agree to
1e-5 with the oracle run in FP64 on the promoted system."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_F32, REL_F64, dev, host, rel_err, say, tie_margin

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jac(gpu):
    import paper_1403_5805_amd as jac
    return jac


def test_c1_parity(jac):
    """n=512 FP64, additive margin, tol 1e-10, cap 1000 (first configuration)."""
    A, Xt, B = synth.c1()
    xo, io = oracle.jacobi(A, B, tol=1e-10, max_iter=1000)
    say("c1 n=512 f64")
    X, info = jac.solve(dev(A), dev(B), tol=1e-10, max_iter=1000)
    assert info["status"] == jac.OK, info
    assert info["kernel"] == 129  # every sweep in one launch, A held in registers
    assert tie_margin(A, B, 1e-10, io["iterations"]) > 1e-6
    assert info["iterations"] == io["iterations"] == 9
    assert rel_err(host(X), xo) <= REL_F64
    assert rel_err(host(X), Xt) <= 1e-10


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (3, 2), (37, 1), (127, 3), (128, 1), (129, 4),
                                 (255, 5), (256, 8), (257, 1), (1000, 2), (1031, 1),
                                 (4099, 1), (3000, 16), (700, 33)])
def test_f64_shapes_parity(jac, n, k):
    """Several tiles plus ragged tails, several right-hand sides (k > 32 uses
    column groups)."""
    A, _, B = synth.dominant(n, k, 1000 + n + k)
    tol = 1e-11
    xo, io = oracle.jacobi(A, B, tol=tol, max_iter=500)
    say("f64 shape", n, k)
    X, info = jac.solve(dev(A), dev(B), tol=tol, max_iter=500)
    assert info["status"] == jac.OK == io["status"]
    if tie_margin(A, B, tol, io["iterations"]) > 1e-6:
        assert info["iterations"] == io["iterations"]
    assert rel_err(host(X), xo) <= REL_F64, (n, k)


@pytest.mark.parametrize("n,k", [(100, 1), (1000, 1), (2053, 1), (512, 4), (333, 16)])
def test_f32_parity(jac, n, k):
    """FP32 system of record (A32, b32) solved in FP64 by the oracle."""
    import torch
    A32, _, B32 = synth.dominant_f32(n, k, 2000 + n, synth.MULTIPLICATIVE, 0.5, 1.0)
    xo, io = oracle.jacobi(A32.astype(np.float64), B32.astype(np.float64), tol=1e-6,
                           max_iter=500)
    say("f32", n, k)
    X, info = jac.solve(dev(A32), dev(B32), tol=1e-6, max_iter=500)
    assert info["status"] == jac.OK
    assert X.dtype == torch.float32
    assert rel_err(host(X), xo) <= REL_F32
    assert abs(info["iterations"] - io["iterations"]) <= 1


@pytest.mark.parametrize("n,k", [(300, 1), (1537, 1), (256, 4)])
def test_bf16_parity(jac, n, k):
    """BF16 A widened to FP32 with FP32 accumulation; the oracle solves the
    promoted BF16 system in FP64."""
    import torch
    A, _, B = synth.dominant(n, k, 3000 + n, synth.MULTIPLICATIVE, 0.5, 1.0)
    Ab = torch.from_numpy(A).to(torch.bfloat16)
    Ap = Ab.to(torch.float64).numpy()
    B32 = B.astype(np.float32)
    xo, io = oracle.jacobi(Ap, B32.astype(np.float64), tol=1e-6, max_iter=500)
    say("bf16", n, k)
    X, info = jac.solve(Ab.cuda(), dev(B32), tol=1e-6, max_iter=500)
    assert info["status"] == jac.OK
    assert rel_err(host(X), xo) <= REL_F32


def test_strided_and_unaligned_lda(jac):
    """A with lda > n (aligned) and an odd lda (rows not 16-byte aligned)."""
    import torch
    n = 777
    A, _, B = synth.dominant(n, 2, 41)
    xo, io = oracle.jacobi(A, B, tol=1e-11, max_iter=300)
    for lda in (n + 1, 800):
        big = torch.zeros((n, lda), dtype=torch.float64)
        big[:, :n] = torch.from_numpy(A)
        Ad = big.cuda()[:, :n]
        say("lda", lda)
        X, info = jac.solve(Ad, dev(B), tol=1e-11, max_iter=300)
        assert info["iterations"] == io["iterations"]
        assert rel_err(host(X), xo) <= REL_F64


def test_l2_norm_parity(jac):
    """Euclidean stopping rule (sec. 2, eq. of sec. 3.1)."""
    A, _, B = synth.dominant(900, 3, 77)
    xo, io = oracle.jacobi(A, B, tol=1e-10, max_iter=300, norm="l2")
    say("l2")
    X, info = jac.solve(dev(A), dev(B), tol=1e-10, max_iter=300, norm="l2")
    assert info["status"] == jac.OK
    if tie_margin(A, B, 1e-10, io["iterations"], norm="l2") > 1e-6:
        assert info["iterations"] == io["iterations"]
    assert rel_err(host(X), xo) <= REL_F64
    # the distance subtracts nearly equal iterates: each entry carries an
    # absolute error of a few ulps of |x|, summed over n*k entries
    slack = 64 * np.finfo(np.float64).eps * np.abs(xo).max() * np.sqrt(xo.size)
    assert abs(info["final_delta"] - io["final_delta"]) <= 1e-6 * io["final_delta"] + slack


def test_cap_and_fixed_iteration_mode(jac):
    """tol = 0 runs exactly L sweeps; L = 0 returns X0 with NOT_CONVERGED."""
    A, _, B = synth.dominant(300, 1, 5)
    for L in (1, 2, 7, 64):
        xo, io = oracle.jacobi(A, B, tol=0.0, max_iter=L)
        say("cap", L)
        X, info = jac.solve(dev(A), dev(B), tol=0.0, max_iter=L)
        assert info["status"] == jac.NOT_CONVERGED and info["iterations"] == L
        assert rel_err(host(X), xo) <= REL_F64
    x0 = np.random.default_rng(0).uniform(-1, 1, size=(300, 1))
    X, info = jac.solve(dev(A), dev(B), dev(x0), tol=1.0, max_iter=0)
    assert info["status"] == jac.NOT_CONVERGED and info["iterations"] == 0
    assert np.array_equal(host(X), x0)
    D = np.diag(np.arange(1.0, 301.0))
    X, info = jac.solve(dev(D), dev(B), tol=0.0, max_iter=9)
    assert info["iterations"] == 9 and info["final_delta"] == 0.0


def test_validation_errors_leave_x_untouched(jac):
    import torch
    A, _, B = synth.dominant(200, 2, 6)
    sentinel = np.full((200, 2), 7.5)
    cases = []
    Z = A.copy(); Z[17, 17] = 0.0; Z[150, 150] = 0.0
    cases.append((Z, B, None, jac.ERR_ZERO_DIAGONAL, 17))
    Z = A.copy(); Z[9, 9] = np.inf; Z[40, 40] = 0.0
    cases.append((Z, B, None, jac.ERR_NONFINITE_INPUT, 9))
    Bn = B.copy(); Bn[123, 1] = np.nan
    cases.append((A, Bn, None, jac.ERR_NONFINITE_INPUT, 123))
    x0 = np.zeros((200, 2)); x0[55, 0] = -np.inf
    cases.append((A, B, x0, jac.ERR_NONFINITE_INPUT, 55))
    for Ai, Bi, x0i, st, bad in cases:
        out = dev(sentinel)
        say("validation", st, bad)
        X, info = jac.solve(dev(Ai), dev(Bi), dev(x0i) if x0i is not None else None, out=out)
        _, io = oracle.jacobi(Ai, Bi, X0=x0i)
        assert info["status"] == st == io["status"]
        assert info["bad_index"] == bad == io["bad_index"]
        assert np.array_equal(host(out), sentinel)
    with pytest.raises(RuntimeError):
        jac.solve(dev(A), dev(B), tol=-1.0, raise_on_error=True)
    X, info = jac.solve(dev(A), dev(B), max_iter=-3)
    assert info["status"] == jac.ERR_INVALID_ARG
    X, info = jac.solve(dev(A), dev(B), mode="refine", sweep_dtype="f32",
                        refine_tol=1e-10)
    assert info["status"] == jac.OK  # FP64 system: refinement is allowed
    # refinement needs an FP64 system: the binding refuses FP32 operands (the
    # library's own check of this is exercised through the raw ABI on the CPU)
    with pytest.raises(TypeError):
        jac.solve(dev(A.astype(np.float32)), dev(B.astype(np.float32)), mode="refine")
    del torch


def test_divergence_of_paper_inputs(jac):
    """The paper's own U[0,1] inputs (sec. 4) are not dominant and overflow."""
    A, b, x0 = synth.paper_uniform(64, 4)
    xo, io = oracle.jacobi(A, b, X0=x0, tol=1e-8, max_iter=10000)
    say("divergence")
    X, info = jac.solve(dev(A), dev(b), dev(x0), tol=1e-8, max_iter=10000)
    assert info["status"] == jac.DIVERGED == io["status"]
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert not np.isfinite(info["final_delta"])


def test_closed_form_family_large_n(jac):
    """A = a I + c (J - I), b = beta 1: exact iterates and stopping sweep known
    in closed form, checked at the full FP32 size n = 16384."""
    import pins
    import torch
    n, a, c, beta, tol = 16384, 40000, 1, 3, 1e-6
    k, s, margin = pins.closed_form(n, a, c, beta, tol)
    assert margin > 1e-3
    A = torch.full((n, n), float(c), dtype=torch.float32, device="cuda")
    A.fill_diagonal_(float(a))
    b = torch.full((n,), float(beta), dtype=torch.float32, device="cuda")
    say("closed form n=16384 f32")
    X, info = jac.solve(A, b, tol=tol, max_iter=100)
    assert info["status"] == jac.OK and info["iterations"] == k
    assert rel_err(host(X), np.full(n, float(s))) <= REL_F32
    n64, a64, c64, beta64, tol64 = 8192, 30000, -1, 2, 1e-12
    k64, s64, m64 = pins.closed_form(n64, a64, c64, beta64, tol64)
    assert m64 > 1e-3
    A = torch.full((n64, n64), float(c64), dtype=torch.float64, device="cuda")
    A.fill_diagonal_(float(a64))
    b = torch.full((n64,), float(beta64), dtype=torch.float64, device="cuda")
    say("closed form n=8192 f64")
    X, info = jac.solve(A, b, tol=tol64, max_iter=100)
    assert info["status"] == jac.OK and info["iterations"] == k64
    assert rel_err(host(X), np.full(n64, float(s64))) <= REL_F64


def test_integer_exact_fixed_point_bitwise(jac):
    """Entries in {-1,0,1}, a_ii = rowsum + 1, integer X_true and X0 = X_true:
    every partial sum is an integer below 2^24, exact in FP32 in any order, so
    Delta_1 = 0 and X = X0 bitwise at n = 16384."""
    import torch
    n = 16384
    g = torch.Generator().manual_seed(7)
    A = torch.randint(-1, 2, (n, n), generator=g, dtype=torch.int8).to(torch.float32)
    A.fill_diagonal_(0.0)
    A += torch.diag(A.abs().sum(dim=1) + 1.0)
    xt = torch.randint(-4, 5, (n,), generator=g).to(torch.float32)
    b = (A.to(torch.float64) @ xt.to(torch.float64)).to(torch.float32)
    say("integer exact n=16384")
    X, info = jac.solve(A.cuda(), b.cuda(), xt.cuda(), tol=1e-30, max_iter=5)
    assert info["iterations"] == 1 and info["final_delta"] == 0.0
    assert torch.equal(X.cpu(), xt)


def test_determinism_and_scaling_bitwise(jac):
    """Two runs are bitwise equal; scaling row i and b_i by 2^e_i leaves every
    iterate bitwise unchanged (component equation: only exponents change)."""
    import torch
    A, _, B = synth.dominant(2049, 2, 99)
    Ad, Bd = dev(A), dev(B)
    say("determinism")
    X1, i1 = jac.solve(Ad, Bd, tol=1e-10, max_iter=200)
    X2, i2 = jac.solve(Ad, Bd, tol=1e-10, max_iter=200)
    assert torch.equal(X1, X2) and i1["iterations"] == i2["iterations"]
    e = np.random.default_rng(1).integers(-30, 31, size=2049)
    s = np.ldexp(1.0, e)
    X3, i3 = jac.solve(dev(A * s[:, None]), dev(B * s[:, None]), tol=1e-10, max_iter=200)
    assert torch.equal(X1, X3) and i1["iterations"] == i3["iterations"]
    assert i1["final_delta"] == i3["final_delta"]


def test_resume_bitwise(jac):
    """The state is (x^k, k): resuming from x^k with cap L - k reproduces the
    uninterrupted run bitwise."""
    import torch
    A, _, B = synth.dominant(1500, 1, 12)
    Ad, Bd = dev(A), dev(B)
    say("resume")
    full, fi = jac.solve(Ad, Bd, tol=0.0, max_iter=12)
    part, _ = jac.solve(Ad, Bd, tol=0.0, max_iter=5)
    rest, ri = jac.solve(Ad, Bd, part.clone(), tol=0.0, max_iter=7)
    assert torch.equal(full, rest) and fi["final_delta"] == ri["final_delta"]


def test_x0_aliases_x(jac):
    A, _, B = synth.dominant(640, 2, 13)
    xo, io = oracle.jacobi(A, B, X0=np.ones((640, 2)), tol=1e-11, max_iter=200)
    X = dev(np.ones((640, 2)))
    say("alias")
    X2, info = jac.solve(dev(A), dev(B), X, out=X, tol=1e-11, max_iter=200)
    assert X2.data_ptr() == X.data_ptr()
    assert info["iterations"] == io["iterations"]
    assert rel_err(host(X), xo) <= REL_F64


def test_c2_full_size_parity(jac):
    """n = 16384 FP32, multiplicative margin U[0.5,1], tol 1e-6 (second
    configuration) against the FP64 oracle on the promoted system; and one sweep
    from a random x0 checked row by row at sampled rows."""
    import torch
    A32, Xt, B32 = synth.c2()
    A64 = A32.astype(np.float64)
    b64 = B32[:, 0].astype(np.float64)
    xo, io = oracle.jacobi(A64, b64, tol=1e-6, max_iter=300)
    Ad, bd = dev(A32), dev(B32[:, 0])
    say("c2 n=16384 f32 natural")
    X, info = jac.solve(Ad, bd, tol=1e-6, max_iter=300)
    assert info["status"] == jac.OK
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert rel_err(host(X), xo) <= REL_F32
    x0 = np.random.default_rng(3).uniform(-1, 1, size=16384).astype(np.float32)
    say("c2 one sweep sampled")
    X1, i1 = jac.solve(Ad, bd, dev(x0), tol=0.0, max_iter=1)
    rows = np.random.default_rng(4).choice(16384, size=256, replace=False)
    want = oracle.update_rows(A32, b64, x0.astype(np.float64), rows)[:, 0]
    got = host(X1)[rows]
    assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()
    del torch


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,k,pad", [(1, 1, 0), (5, 2, 0), (37, 2, 1), (512, 1, 0),
                                     (1000, 2, 3), (1500, 1, 0), (2048, 1, 0), (2048, 2, 1),
                                     (3000, 1, 1)])
def test_small_system_kernel(jac, monkeypatch, dtype, n, k, pad):
    """Systems of at most 2048 rows (one or two right-hand sides) run every
    sweep in one persistent launch, the small-system kernel; the per-sweep
    vector kernel (JACOBI_SMALL_MAX=0) gives the same count and X to
    rounding, and both agree with the oracle (FP64 to 1e-12 with the oracle's
    count when the tie margin holds; FP32 and BF16 A to 1e-5 with the oracle
    run in FP64 on the promoted system).  Rows that are not 16-byte aligned
    (odd leading dimension) included; the Euclidean norm and the cap too."""
    import torch
    if dtype == "f64":
        A, _, B = synth.dominant(n, k, 5100 + n + k)
        Ap, Bp, tol, bar = A, B, 1e-11, REL_F64
        tdt, vdt = torch.float64, torch.float64
    else:
        A32, _, B32 = synth.dominant_f32(n, k, 5100 + n + k, synth.ADDITIVE, 1.0, 2.0)
        Ap = (torch.from_numpy(A32).to(torch.bfloat16).to(torch.float64).numpy()
              if dtype == "bf16" else A32.astype(np.float64))
        A, B, Bp, tol, bar = A32, B32, B32.astype(np.float64), 1e-6, REL_F32
        tdt, vdt = (torch.bfloat16 if dtype == "bf16" else torch.float32), torch.float32
    big = torch.zeros((n, n + pad), dtype=torch.float64)
    big[:, :n] = torch.from_numpy(np.asarray(A, dtype=np.float64))
    Ad = big.to(tdt).cuda()[:, :n]
    Bd = torch.from_numpy(np.asarray(B)).to(vdt).cuda()
    xo, io = oracle.jacobi(Ap, Bp, tol=tol, max_iter=500)
    out = {}
    for mode in ("small", "lds", "vector"):
        # every size of this test fits the small kernel's LDS: force it (the
        # register-resident variant where the rows fit, else the LDS one), or
        # force its LDS variant, or turn it off
        monkeypatch.setenv("JACOBI_SMALL_MAX", "0" if mode == "vector" else "4096")
        monkeypatch.setenv("JACOBI_SMALL_REG", "0" if mode == "lds" else "1")
        say("small-system kernel", dtype, n, k, pad, mode)
        out[mode] = (jac.solve(Ad, Bd, tol=tol, max_iter=500),
                     jac.solve(Ad, Bd, tol=0.0, max_iter=7, norm="l2"))
    monkeypatch.delenv("JACOBI_SMALL_REG")
    (Xs, inf_s), (Ls, linf_s) = out["small"]
    (Xd, inf_d), (Ld, linf_d) = out["lds"]
    (Xv, inf_v), (Lv, linf_v) = out["vector"]
    assert inf_s["kernel"] in (128, 129) and inf_d["kernel"] == 128 and inf_v["kernel"] == 0
    # the rows of every wave fit its registers (12 pieces of 16 bytes per lane
    # and row for FP64 n = 1500 and FP32 n = 3000) except for FP64 n = 2048,
    # k = 2 and FP64 n = 3000
    assert (inf_s["kernel"] == 129) == (not (dtype == "f64" and (n, k) in ((2048, 2), (3000, 1))))
    # both variants take the same products in the same order: the same bits
    # (the Euclidean distance adds one partial sum per workgroup, and the
    # variants differ in workgroup count: equal to rounding)
    assert torch.equal(Xs, Xd) and inf_s["iterations"] == inf_d["iterations"]
    assert inf_s["final_delta"] == inf_d["final_delta"]
    assert torch.equal(Ls, Ld)
    assert abs(linf_s["final_delta"] - linf_d["final_delta"]) <= 1e-13 * linf_d["final_delta"]
    assert inf_s["status"] == inf_v["status"] == jac.OK, (inf_s, inf_v)
    assert abs(inf_s["iterations"] - inf_v["iterations"]) <= (0 if dtype == "f64" else 1)
    if dtype == "f64" and tie_margin(A, B, tol, io["iterations"]) > 1e-6:
        assert inf_s["iterations"] == io["iterations"], (inf_s, io)
    assert rel_err(host(Xs), xo) <= bar and rel_err(host(Xv), xo) <= bar
    assert linf_s["iterations"] == linf_v["iterations"] == 7
    assert linf_s["status"] == jac.NOT_CONVERGED
    # the distance is a difference of consecutive iterates: it carries the
    # iterate's absolute rounding, so it is compared at the X bar times max|x|
    xm = float(np.abs(host(Ls)).max())
    assert abs(linf_s["final_delta"] - linf_v["final_delta"]) <= bar * xm
    xl, _ = oracle.jacobi(Ap, Bp, tol=0.0, max_iter=7, norm="l2")
    assert rel_err(host(Ls), xl) <= bar
    # the same inputs give the same bits again
    monkeypatch.setenv("JACOBI_SMALL_MAX", "4096")
    X2, inf2 = jac.solve(Ad, Bd, tol=tol, max_iter=500)
    assert torch.equal(X2, Xs) and inf2["iterations"] == inf_s["iterations"]
    # the fused launch (set-up, checks and copy-out in the register kernel,
    # outcome written to the host) equals the separate set-up, read-back and
    # copy-out bitwise, from zero and from a given X0, over 3 sweeps and to tol
    x0 = torch.from_numpy(np.random.default_rng(n + k).uniform(-1, 1, size=(n, k))).to(vdt).cuda()
    got = {}
    for fz in ("1", "0"):
        monkeypatch.setenv("JACOBI_SMALL_FUSED", fz)
        say("small-system kernel fused", fz, dtype, n, k, pad)
        got[fz] = [jac.solve(Ad, Bd, x, tol=t, max_iter=m)
                   for x in (None, x0) for t, m in ((tol, 500), (0.0, 3))]
    monkeypatch.delenv("JACOBI_SMALL_FUSED")
    # four and eight waves per workgroup (where both exist): the same bits
    for wv in ("4", "8"):
        monkeypatch.setenv("JACOBI_SMALL_WAVES", wv)
        say("small-system kernel waves", wv, dtype, n, k, pad)
        Xw, iw = jac.solve(Ad, Bd, tol=tol, max_iter=500)
        assert torch.equal(Xw, Xs) and iw["iterations"] == inf_s["iterations"], (wv, dtype, n, k)
        assert iw["final_delta"] == inf_s["final_delta"]
    monkeypatch.delenv("JACOBI_SMALL_WAVES")
    for (Xf, i_f), (Xu, i_u) in zip(got["1"], got["0"]):
        assert i_f["kernel"] == i_u["kernel"] == inf_s["kernel"]
        assert torch.equal(Xf, Xu), (dtype, n, k)
        assert (i_f["status"], i_f["iterations"], i_f["final_delta"]) == \
            (i_u["status"], i_u["iterations"], i_u["final_delta"])
    monkeypatch.delenv("JACOBI_SMALL_MAX")


def test_stream_probe(jac):
    """The achievable-read probe: a rate between a fraction of the published
    HBM peak and a little above it on a buffer larger than the caches, the
    buffer unchanged, bad arguments refused."""
    import torch
    buf = torch.arange(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
    ref = buf.clone()
    say("stream probe")
    p = jac.stream_probe(buf, reps=2)
    assert 1000.0 < p["GBps"] < 8800.0, p
    assert p["wg_per_cu"] in (2, 4, 8, 16)
    assert torch.equal(buf, ref)
    with pytest.raises(ValueError):
        jac.stream_probe(buf[::2])
    with pytest.raises(RuntimeError):
        jac.stream_probe(buf[:1], reps=1)  # 4 bytes: below one 16-byte piece


def test_small_fused_launches_in_a_row(jac, monkeypatch):
    """Fused small-system solves one after another on one context, each
    continuing the barrier count and slot rotation the previous launch left
    (no k_init_ctl between them): different sizes, dtypes, k, norms and caps,
    with an invalid input and a refinement solve (which re-initialise the
    control block) in between, the whole sequence twice.  Every result equals
    the same solve with the separate set-up (JACOBI_SMALL_FUSED=0) bitwise."""
    import torch
    ctx = jac.Context(0)
    cases = []
    for n, k, seed in ((512, 1, 1), (200, 2, 2), (37, 1, 3), (1254, 2, 4)):
        A, _, B = synth.dominant(n, k, 6100 + seed)
        cases.append(("f64", dev(A), dev(B)))
    for n, k, seed, dt in ((1000, 1, 5, torch.float32), (2048, 2, 6, torch.bfloat16)):
        A, _, B = synth.dominant_f32(n, k, 6100 + seed, synth.ADDITIVE, 1.0, 2.0)
        cases.append(("f32" if dt == torch.float32 else "bf16",
                      torch.from_numpy(A).to(dt).cuda(), torch.from_numpy(B).cuda()))
    opts = [dict(tol=1e-10, max_iter=500), dict(tol=0.0, max_iter=5, norm="l2"),
            dict(tol=0.0, max_iter=1), dict(tol=1e-11, max_iter=500, norm="l2"),
            dict(tol=1e-6, max_iter=500), dict(tol=1e-6, max_iter=4)]
    Az, _, Bz = synth.dominant(300, 1, 6107)
    Az[123, 123] = 0.0
    Ar, _, Br = synth.dominant(256, 1, 6108)

    def sequence():
        out = []
        for rep in range(2):
            for i, ((dt, Ad, Bd), o) in enumerate(zip(cases, opts)):
                say("fused chain", rep, i, dt, tuple(Ad.shape), Bd.shape[1])
                out.append(jac.solve(Ad, Bd, ctx=ctx, **o))
                if i == 2:
                    out.append(jac.solve(dev(Az), dev(Bz), ctx=ctx))
                if i == 3:
                    out.append(jac.solve(dev(Ar), dev(Br), ctx=ctx, mode="refine",
                                         sweep_dtype="f32", refine_tol=1e-12))
        return out
    fused = sequence()
    monkeypatch.setenv("JACOBI_SMALL_FUSED", "0")
    sep = sequence()
    monkeypatch.delenv("JACOBI_SMALL_FUSED")
    for (Xf, i_f), (Xs, i_s) in zip(fused, sep):
        assert (i_f["status"], i_f["iterations"], i_f["final_delta"], i_f["bad_index"]) == \
            (i_s["status"], i_s["iterations"], i_s["final_delta"], i_s["bad_index"])
        if i_f["status"] >= 0:
            assert torch.equal(Xf, Xs)
    assert [i["status"] for _, i in fused].count(jac.ERR_ZERO_DIAGONAL) == 2
    # every case ran fused in the register kernel, twice (FP64 n = 1254, k = 2
    # with 12 pieces of 16 bytes per lane and row)
    assert [i["kernel"] for _, i in fused].count(129) == 12
    # X written from registers into a strided view (ldx = k + 3), with X0
    # absent (fused) and given with that leading dimension (separate set-up)
    A, _, B = synth.dominant(300, 2, 6109)
    Ad, Bd = dev(A), dev(B)
    ref, iref = jac.solve(Ad, Bd, ctx=ctx, tol=1e-10, max_iter=500)
    for x0 in (None, torch.zeros((300, 5), dtype=torch.float64, device="cuda")[:, :2]):
        say("fused strided out", x0 is None)
        big = torch.full((300, 5), 7.5, dtype=torch.float64, device="cuda")
        X, info = jac.solve(Ad, Bd, x0, out=big[:, :2], ctx=ctx, tol=1e-10, max_iter=500)
        assert info["kernel"] == 129 and info["iterations"] == iref["iterations"]
        assert torch.equal(big[:, :2], ref) and bool((big[:, 2:] == 7.5).all())
    ctx.close()
