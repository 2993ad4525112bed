"""GPU test of the no-allocation entry point jacobi_solve_noalloc (called
through the C ABI by the binding's solve_noalloc): X, count, status and
distance equal jacobi_solve's bitwise, on two calls in a row where the second
is smaller (the fixed workspace keeps the previous call's contents), with no
change in the device's free memory across calls; shapes above the fixed
workspace and options outside the vector path are refused before any device
work."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import synth
from gpu_util import dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jac(gpu):
    import paper_1403_5805_amd as jac
    return jac


def _case(n, k, dtype, seed, pad=0, x0=False):
    import torch
    A, Xt, B = synth.dominant(n, k, seed, synth.ADDITIVE, 1.0, 2.0)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    vdt = torch.float64 if dtype == "f64" else torch.float32
    big = torch.zeros((n, n + pad), dtype=tdt)
    big[:, :n] = torch.from_numpy(A).to(tdt)
    Ad = big.cuda()[:, :n]
    Bd = torch.from_numpy(B).to(vdt).cuda()
    X0 = None
    if x0:
        X0 = torch.from_numpy(np.random.default_rng(seed).uniform(-1, 1, (n, k))).to(vdt).cuda()
    return Ad, Bd, X0


def _same(jac, case, **opts):
    """Run the no-allocation entry point then jacobi_solve on one case and
    compare them bitwise; returns the no-allocation call's info."""
    import torch
    Ad, Bd, X0 = case
    out_na = torch.empty_like(Bd)
    out_ref = torch.empty_like(Bd)
    free0 = torch.cuda.mem_get_info()[0]
    Xn, ina = jac.solve_noalloc(Ad, Bd, X0, out=out_na, **opts)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    Xr, iref = jac.solve(Ad, Bd, X0, out=out_ref, **opts)
    assert ina["status"] == iref["status"], (ina, iref)
    assert ina["status"] in (jac.OK, jac.NOT_CONVERGED), ina
    for key in ("iterations", "final_delta", "bad_index"):
        assert ina[key] == iref[key], (key, ina, iref)
    assert torch.equal(Xn, Xr)
    return ina, free0, free1


@pytest.mark.parametrize("first,second", [
    ((1536, 2, "f64", 11, 0, False), (300, 1, "f64", 12, 0, False)),
    ((2001, 2, "f32", 13, 1, True), (97, 1, "f32", 14, 1, False)),
    ((1200, 1, "bf16", 15, 0, False), (64, 2, "bf16", 16, 1, True)),
])
def test_noalloc_matches_solve_twice(jac, first, second):
    """Two calls in a row (the second smaller) equal jacobi_solve bitwise; the
    free device memory does not move across the second call (the first may
    load the code object that holds the workspace)."""
    say("noalloc first", first)
    a = _case(*first)
    _same(jac, a, tol=1e-10, max_iter=500)
    say("noalloc second", second)
    b = _case(*second)
    info, free0, free1 = _same(jac, b, tol=1e-10, max_iter=500)
    assert free0 == free1, (free0, free1)
    # L2 norm and a fixed-sweep run on the same buffers
    say("noalloc second l2", second)
    _same(jac, b, tol=0.0, max_iter=7, norm="l2")


def test_noalloc_validation_and_edges(jac):
    """A zero diagonal is reported with its row and leaves X untouched;
    max_iter = 0 returns X0."""
    import torch
    Ad, Bd, X0 = _case(257, 2, "f64", 21, x0=True)
    Z = Ad.clone()
    Z[100, 100] = 0.0
    out = torch.full_like(Bd, 7.0)
    say("noalloc zero diagonal")
    _, info = jac.solve_noalloc(Z, Bd, out=out)
    assert info["status"] == jac.ERR_ZERO_DIAGONAL and info["bad_index"] == 100
    assert bool((out == 7.0).all())
    say("noalloc max_iter 0")
    X, info = jac.solve_noalloc(Ad, Bd, X0, max_iter=0)
    assert info["status"] == jac.NOT_CONVERGED and info["iterations"] == 0
    assert torch.equal(X, X0)


def test_noalloc_refuses_before_device_work(jac):
    """Shapes whose workspace exceeds the fixed array, k > 2, refinement and
    per-sweep profiling are refused with ERR_INVALID_ARG before any device
    work (the device pointers of a small case stand in for the large one:
    nothing is read)."""
    from paper_1403_5805_amd import _lib
    lib = _lib.load()
    Ad, Bd, _ = _case(64, 1, "f64", 31)
    o = jac.make_options()
    info = _lib.Info()
    p = ctypes.c_void_p
    say("noalloc refusals")
    n = 700000  # F64, k = 2: about 30 MB of workspace
    st = lib.jacobi_solve_noalloc(n, 2, jac.F64, p(Ad.data_ptr()), n, p(Bd.data_ptr()), 2, None,
                                  p(Bd.data_ptr()), 2, ctypes.byref(o), None, ctypes.byref(info))
    assert st == jac.ERR_INVALID_ARG and "workspace" in jac.last_error()
    for kw in ({"mode": "refine"}, {"profile": True}):
        o = jac.make_options(**kw)
        st = lib.jacobi_solve_noalloc(64, 1, jac.F64, p(Ad.data_ptr()), 64, p(Bd.data_ptr()), 1,
                                      None, p(Bd.data_ptr()), 1, ctypes.byref(o), None,
                                      ctypes.byref(info))
        assert st == jac.ERR_INVALID_ARG, kw
    o = jac.make_options()
    st = lib.jacobi_solve_noalloc(64, 3, jac.F64, p(Ad.data_ptr()), 64, p(Bd.data_ptr()), 3, None,
                                  p(Bd.data_ptr()), 3, ctypes.byref(o), None, ctypes.byref(info))
    assert st == jac.ERR_INVALID_ARG
