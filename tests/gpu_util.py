"""Helpers shared by the GPU parity tests (marshalling and error measures)."""
from __future__ import annotations

import sys

import numpy as np

REL_F64 = 1e-12   # FP64 sweeps vs the FP64 oracle, norm-wise relative
REL_F32 = 1e-5    # FP32 (and BF16-A / FP32-accumulate) sweeps vs the FP64 oracle
REL_REFINE = 1e-10


def say(*a):
    """Name the case before each GPU step, flushed, so a crash log shows it."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t) -> np.ndarray:
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def rel_err(x, ref) -> float:
    """Norm-wise relative error ||x - ref||_inf / ||ref||_inf."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    if den == 0:
        return float(np.abs(x).max())
    return float(np.abs(x - ref).max() / den)


def tie_margin(A, B, tol, k_stop, norm="inf"):
    """min |Delta_k - tol| / tol over the last two sweeps of an oracle run,
    recomputed from the oracle's own iterates.  Count parity is only claimed
    when this exceeds 1e-6."""
    import oracle
    ds = []
    for L in range(max(1, k_stop - 2), k_stop + 1):
        x1, _ = oracle.jacobi(A, B, tol=0.0, max_iter=L, norm=norm)
        x0, _ = oracle.jacobi(A, B, tol=0.0, max_iter=L - 1, norm=norm)
        d = np.asarray(x1) - np.asarray(x0)
        ds.append(np.abs(d).max() if norm == "inf" else np.linalg.norm(d))
    return min(abs(d - tol) / tol for d in ds[-2:])
