"""GPU tests of the serving engine (jacobi_serve_*): results against the FP64
oracle's tight solution, bitwise equality alone vs in the mix, admission by
HBM budget, input errors, and shutdown with requests in flight."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_REFINE, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jac(gpu):
    import paper_1403_5805_amd as jac
    return jac


def _requests():
    shapes = [(200, 1, "bf16"), (777, 4, "f32"), (1500, 16, "bf16"), (333, 1, "f32"),
              (1024, 4, "bf16"), (129, 16, "f32")]
    reqs = []
    for i, (n, k, lo) in enumerate(shapes):
        A, Xt, B = synth.dominant(n, k, 7000 + i, synth.MULTIPLICATIVE, 0.2, 1.0)
        reqs.append((A, B, lo))
    return reqs


def test_served_results_match_oracle(jac):
    reqs = _requests()
    srv = jac.Server(max_active=8)
    say("serve mix")
    tickets = []
    for A, B, lo in reqs:
        t, st = srv.submit(A, B, sweep_dtype=lo)
        assert st == 0
        tickets.append(t)
    for (A, B, lo), t in zip(reqs, tickets):
        X, info = srv.wait(t, timeout_s=120)
        assert info["status"] == jac.OK, info
        xr, _ = oracle.jacobi(A, B, tol=1e-15, max_iter=1000)
        assert rel_err(X, xr) <= REL_REFINE
        assert info["rel_residual"] < 1e-12 and info["outer_iterations"] >= 2
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    assert st["hbm_in_use"] == 0 and st["hbm_peak"] > 0
    srv.close()


def test_alone_and_in_mix_bitwise(jac):
    """Each result is the same alone and in the mix (continuous batching never
    changes a request's arithmetic)."""
    reqs = _requests()
    srv = jac.Server(max_active=16)
    say("serve mix vs alone")
    mixed = [srv.submit(A, B, sweep_dtype=lo)[0] for A, B, lo in reqs]
    mix_out = [srv.wait(t, timeout_s=120) for t in mixed]
    for (A, B, lo), (Xm, im) in zip(reqs, mix_out):
        t, _ = srv.submit(A, B, sweep_dtype=lo)
        Xa, ia = srv.wait(t, timeout_s=120)
        assert np.array_equal(Xa, Xm)
        assert ia["iterations"] == im["iterations"]
        assert ia["outer_iterations"] == im["outer_iterations"]
    srv.close()


def test_admission_rejection_and_errors(jac):
    """A request that can never fit the budget is rejected; one that fits runs
    even though the budget holds only one request at a time; a zero diagonal
    is reported with its row."""
    A, Xt, B = synth.dominant(300, 2, 7100, synth.MULTIPLICATIVE, 0.2, 1.0)
    big, _, bigb = synth.dominant(1200, 1, 7101, synth.MULTIPLICATIVE, 0.2, 1.0)
    srv = jac.Server(max_active=4, hbm_budget_bytes=4 * 1024 * 1024)
    say("serve admission")
    t, st = srv.submit(big, bigb)
    assert st == jac.ERR_REJECTED
    _, info = srv.poll(t)
    assert info["status"] == jac.ERR_REJECTED
    ts = [srv.submit(A, B, sweep_dtype="f32")[0] for _ in range(3)]
    for t in ts:
        X, info = srv.wait(t, timeout_s=120)
        assert info["status"] == jac.OK
    st = srv.stats()
    assert st["hbm_peak"] <= 4 * 1024 * 1024
    Z = A.copy(); Z[41, 41] = 0.0
    t, st = srv.submit(Z, B)
    assert st == jac.ERR_ZERO_DIAGONAL
    _, info = srv.poll(t)
    assert info["bad_index"] == 41
    # a per-request cap on the refinement steps: stopped after its own cap, while
    # the same request under the server's cap converges
    t, st = srv.submit(A, B, sweep_dtype="bf16", rel_tol=1e-12, max_outer=1)
    assert st == 0
    X, info = srv.wait(t, timeout_s=120)
    assert info["status"] == jac.NOT_CONVERGED and info["outer_iterations"] == 2, info
    t, st = srv.submit(A, B, sweep_dtype="bf16", rel_tol=1e-12)
    X, info = srv.wait(t, timeout_s=120)
    assert info["status"] == jac.OK and info["outer_iterations"] > 2, info
    t, st = srv.submit(A, B, max_outer=-1)
    assert st == jac.ERR_INVALID_ARG
    srv.close()


def test_shutdown_with_requests_in_flight(jac):
    """Destroying the server with work queued returns promptly; requests that
    never finished leave their output untouched."""
    A, Xt, B = synth.dominant(1024, 1, 7200, synth.MULTIPLICATIVE, 0.2, 1.0)
    srv = jac.Server(max_active=1)
    outs = [np.full((1024, 1), 5.0) for _ in range(12)]
    say("serve shutdown")
    for o in outs:
        srv.submit(A, B, out=o)
    srv.close()
    untouched = sum(1 for o in outs if np.all(o == 5.0))
    done = [o for o in outs if not np.all(o == 5.0)]
    assert untouched >= 1
    xr, _ = oracle.jacobi(A, B, tol=1e-15, max_iter=1000)
    for o in done:
        assert rel_err(o, xr) <= REL_REFINE


def test_served_large_requests_match_oracle(jac):
    """Requests at the large end of the serving mix (n up to 16384, k = 1, 4
    and 16, FP32 and BF16 inner sweeps), served together with the small mix:
    large FP64 residual jobs, several arena slabs and inner solves of
    different sizes in one batched launch.  Each result is compared with the
    oracle's tight solution x_ref (computed in threads while the server runs)
    at the refinement bar."""
    import concurrent.futures as cf
    shapes = [(16384, 4, "bf16"), (9001, 16, "f32"), (8192, 16, "bf16"), (12289, 1, "f32")]
    big = []
    for i, (n, k, lo) in enumerate(shapes):
        A, Xt, B = synth.dominant(n, k, 7300 + i, synth.MULTIPLICATIVE, 0.2, 1.0)
        big.append((A, B, lo))
    reqs = big + _requests()
    srv = jac.Server(max_active=16)
    say("serve large", [s[:2] for s in shapes])
    tickets = [srv.submit(A, B, sweep_dtype=lo)[0] for A, B, lo in reqs]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        refs = list(ex.map(lambda r: oracle.jacobi(r[0], r[1], tol=1e-15, max_iter=1000)[0],
                           big))
    for idx, ((A, B, lo), t) in enumerate(zip(reqs, tickets)):
        X, info = srv.wait(t, timeout_s=120)
        assert info["status"] == jac.OK, (idx, info)
        assert info["rel_residual"] < 1e-12
        if idx < len(big):
            err = rel_err(X, refs[idx])
            print(f"served n={A.shape[0]} k={B.shape[1]} {lo}: err={err:.2e} "
                  f"outer={info['outer_iterations']} inner={info['iterations']}", flush=True)
            assert err <= REL_REFINE, (idx, err)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["hbm_in_use"] == 0
    srv.close()
