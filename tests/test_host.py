"""CPU tests of the C ABI and the host logic (no GPU, no compute calls).

* libjacobi.so loads and exports exactly the entry points include/jacobi.h
  declares;
* the ctypes structures and constants of the Python binding match the
  header's layouts and enum values (checked by a gcc-built probe of the header);
* defaults, status strings and argument validation that returns before any
  device work;
* the Python binding refuses host tensors (there is no CPU path) and fails
  loudly without the library; the package never imports the oracle;
* the batched kernel's workgroup planner keeps its guarantees (every row
  covered once, grid within the resident capacity, split systems alone on
  their workgroups) on random size mixes.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jacobi.h")
PKG = os.path.join(ROOT, "paper_1403_5805_amd")
LIB = os.path.join(PKG, "libjacobi.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, os.path.join(PKG, "build.py")], check=True)
    from paper_1403_5805_amd import _lib
    return _lib.load()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^JACOBI_API [^(]*?\b(jacobi_\w+)\(", text, re.M)))


def test_exports_match_header(lib):
    declared = _declared()
    assert len(declared) == 20
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], check=True, capture_output=True,
                         text=True).stdout
    exported = sorted(ln.split()[-1] for ln in out.splitlines() if " T " in ln)
    assert exported == declared
    for name in declared:
        assert hasattr(lib, name)


_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "jacobi.h"
#define F(T, m) printf(#T " " #m " %zu %zu\n", offsetof(T, m), sizeof(((T*)0)->m));
#define S(T) printf(#T " sizeof %zu 0\n", sizeof(T));
int main(void) {
@STRUCTS@
    printf("enum JACOBI_OK %d\n", JACOBI_OK);
@ENUMS@
    return 0;
}
"""


def _c_layouts(tmp_path, structs, enums):
    body = []
    for cname, fields in structs.items():
        body.append(f"    S({cname})")
        for f in fields:
            body.append(f"    F({cname}, {f})")
    en = [f'    printf("enum {e} %d\\n", (int){e});' for e in enums]
    src = tmp_path / "probe.c"
    src.write_text(_PROBE.replace("@STRUCTS@", "\n".join(body)).replace("@ENUMS@",
                                                                        "\n".join(en)))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lay, ev = {}, {}
    for ln in out.splitlines():
        parts = ln.split()
        if parts[0] == "enum":
            ev[parts[1]] = int(parts[2])
        else:
            lay[(parts[0], parts[1])] = (int(parts[2]), int(parts[3]))
    return lay, ev


def test_struct_layouts_and_enums_match_binding(tmp_path):
    from paper_1403_5805_amd import _lib
    pairs = {"jacobi_options": _lib.Options, "jacobi_info": _lib.Info,
             "jacobi_system": _lib.System, "jacobi_serve_config": _lib.ServeConfig,
             "jacobi_request": _lib.Request, "jacobi_serve_stats": _lib.ServeStats}
    structs = {c: [f for f, _ in py._fields_] for c, py in pairs.items()}
    enums = ["JACOBI_NOT_CONVERGED", "JACOBI_DIVERGED", "JACOBI_PENDING", "JACOBI_CANCELLED",
             "JACOBI_ERR_INVALID_ARG", "JACOBI_ERR_ZERO_DIAGONAL",
             "JACOBI_ERR_NONFINITE_INPUT", "JACOBI_ERR_OUT_OF_MEMORY", "JACOBI_ERR_DEVICE",
             "JACOBI_ERR_REJECTED", "JACOBI_ERR_INTERNAL", "JACOBI_F64", "JACOBI_F32",
             "JACOBI_BF16", "JACOBI_NORM_INF", "JACOBI_NORM_L2", "JACOBI_MODE_PLAIN",
             "JACOBI_MODE_REFINE"]
    lay, ev = _c_layouts(tmp_path, structs, enums)
    for cname, py in pairs.items():
        assert lay[(cname, "sizeof")][0] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            desc = getattr(py, f)
            assert lay[(cname, f)] == (desc.offset, desc.size), (cname, f)
    for e in enums:
        assert getattr(_lib, e[len("JACOBI_"):]) == ev[e], e


def test_defaults(lib):
    from paper_1403_5805_amd import _lib
    o = _lib.Options()
    lib.jacobi_options_default(ctypes.byref(o))
    assert (o.tol, o.max_iter, o.norm, o.mode) == (1e-8, 10000, _lib.NORM_INF, _lib.MODE_PLAIN)
    assert (o.sweep_dtype, o.inner_rel_tol, o.max_inner, o.max_outer) == (_lib.BF16, 1e-3,
                                                                          200, 50)
    assert (o.refine_tol, o.sync_every, o.profile) == (1e-12, 0, 0)
    c = _lib.ServeConfig()
    lib.jacobi_serve_config_default(ctypes.byref(c))
    assert (c.device, c.max_active, c.hbm_budget_bytes, c.inner_max, c.max_outer) == (
        0, 64, 0, 64, 50)
    assert c.inner_rel_tol == 1e-3


def test_status_strings(lib):
    import paper_1403_5805_amd as jac
    names = {jac.OK: "OK", jac.NOT_CONVERGED: "NOT_CONVERGED", jac.DIVERGED: "DIVERGED",
             jac.PENDING: "PENDING", jac.CANCELLED: "CANCELLED",
             jac.ERR_INVALID_ARG: "ERR_INVALID_ARG", jac.ERR_ZERO_DIAGONAL: "ERR_ZERO_DIAGONAL",
             jac.ERR_NONFINITE_INPUT: "ERR_NONFINITE_INPUT",
             jac.ERR_OUT_OF_MEMORY: "ERR_OUT_OF_MEMORY", jac.ERR_DEVICE: "ERR_DEVICE",
             jac.ERR_REJECTED: "ERR_REJECTED", jac.ERR_INTERNAL: "ERR_INTERNAL"}
    for code, name in names.items():
        assert jac.status_string(code) == name
    assert jac.status_string(12345) == "UNKNOWN"


def _solve_raw(lib, n, k, dt, A, lda, B, ldb, X, ldx, opt=None):
    from paper_1403_5805_amd import _lib
    info = _lib.Info()
    st = lib.jacobi_solve(None, n, k, dt, A, lda, B, ldb, None, X, ldx,
                          ctypes.byref(opt) if opt is not None else None, None,
                          ctypes.byref(info))
    return st, info


def test_invalid_arguments_rejected_before_device_work(lib):
    """Bad sizes, pointers, dtypes and options return ERR_INVALID_ARG from the
    argument checks, before a context or any device memory is touched (the
    non-null pointers below are never dereferenced)."""
    import paper_1403_5805_amd as jac
    from paper_1403_5805_amd import _lib
    p = ctypes.c_void_p(0x1000)
    bad = [
        (0, 1, jac.F64, p, 1, p, 1, p, 1),      # n = 0
        (4, 0, jac.F64, p, 4, p, 1, p, 1),      # k = 0
        (4, 1, jac.F64, p, 3, p, 1, p, 1),      # lda < n
        (4, 2, jac.F64, p, 4, p, 1, p, 2),      # ldb < k
        (4, 2, jac.F64, p, 4, p, 2, p, 1),      # ldx < k
        (4, 1, jac.F64, None, 4, p, 1, p, 1),   # null A
        (4, 1, jac.F64, p, 4, None, 1, p, 1),   # null B
        (4, 1, jac.F64, p, 4, p, 1, None, 1),   # null X
        (4, 1, 7, p, 4, p, 1, p, 1),            # unknown dtype
        (4, 5000, jac.F64, p, 4, p, 5000, p, 5000),  # k beyond 4096
    ]
    for args in bad:
        st, info = _solve_raw(lib, *args)
        assert st == jac.ERR_INVALID_ARG and info.status == st, args
        assert jac.last_error()
    for field, value in [("tol", -1.0), ("tol", float("nan")), ("max_iter", -1), ("norm", 5),
                         ("mode", 9), ("sync_every", -2)]:
        o = jac.make_options()
        setattr(o, field, value)
        st, _ = _solve_raw(lib, 4, 1, jac.F64, p, 4, p, 1, p, 1, o)
        assert st == jac.ERR_INVALID_ARG, field
    o = jac.make_options(mode="refine")
    st, _ = _solve_raw(lib, 4, 1, jac.F32, p, 4, p, 1, p, 1, o)
    assert st == jac.ERR_INVALID_ARG and "REFINE" in jac.last_error()

    infos = (_lib.Info * 1)()
    assert lib.jacobi_solve_batched(None, -1, None, jac.F32, None, None, infos) == \
        jac.ERR_INVALID_ARG
    sysarr = (_lib.System * 1)()
    o = jac.make_options(mode="refine")
    assert lib.jacobi_solve_batched(None, 1, sysarr, jac.F32, ctypes.byref(o), None,
                                    infos) == jac.ERR_INVALID_ARG
    assert infos[0].status == jac.ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.jacobi_serve_create(None, None) == jac.ERR_INVALID_ARG
    assert lib.jacobi_ctx_create(0, None) == jac.ERR_INVALID_ARG
    del h


def test_binding_refuses_host_tensors(lib):
    """The product path has no CPU fallback: host tensors are refused before
    the library is called."""
    import torch

    import paper_1403_5805_amd as jac
    A = torch.eye(4, dtype=torch.float64)
    b = torch.ones(4, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        jac.solve(A, b)
    with pytest.raises(ValueError, match="GPU tensor"):
        jac.solve_batched([(A.float(), b.float())])
    with pytest.raises(ValueError, match="GPU tensor"):
        jac.Batch([(A.float(), b.float())])
    assert jac.Batch([]).solve() == ([], [])
    with pytest.raises(TypeError):
        jac.solve(A.to(torch.int32), b)
    with pytest.raises(ValueError):
        jac.solve(torch.ones(4, 3, dtype=torch.float64), b)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1403_5805_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libjacobi.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.load()


def test_package_does_not_use_the_oracle():
    code = ("import sys; import paper_1403_5805_amd, paper_1403_5805_amd.serve, "
            "paper_1403_5805_amd.batched; "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, check=True,
                         capture_output=True, text=True).stdout.strip()
    assert out == "False"
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "jacobi_oracle" not in text, f


# ---- batched workgroup planner ---------------------------------------------

@pytest.fixture(scope="module")
def plan_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    exe = d / "plan_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(PKG, "csrc", "plan.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def _plan(exe, ns, capacity, tpp=2, unroll=4, bw=64):
    inp = f"{capacity} {tpp} {unroll} {bw} {len(ns)} " + " ".join(str(int(v)) for v in ns)
    out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout
    grid, nwg, wgs, queue = 0, {}, {}, []
    for ln in out.splitlines():
        p = ln.split()
        if p[0] == "grid":
            grid = int(p[1])
        elif p[0] == "nwg":
            nwg[int(p[1])] = int(p[2])
        elif p[0] == "q":
            queue.append(int(p[1]))
        else:
            g, s, r, r0, r1 = map(int, p[1:])
            wgs.setdefault(g, []).append((s, r, r0, r1))
    return grid, nwg, wgs, queue


def _check_plan(ns, capacity, grid, nwg, wgs, queue):
    assert 0 <= grid <= capacity
    assert all(0 <= g < grid for g in wgs)
    if len(wgs) < grid:
        assert queue, "a workgroup without fixed jobs only serves the queue"
    rows = {i: [] for i in range(len(ns))}
    ranks = {i: [] for i in range(len(ns))}
    for g, jobs in wgs.items():
        for s, r, r0, r1 in jobs:
            rows[s].append((r0, r1))
            ranks[s].append(r)
            assert r0 % 16 == 0 and r0 < r1 <= ns[s]
            assert nwg[s] >= 2, "fixed jobs are shares of split systems"
            assert len(jobs) == 1, "a split system's workgroup holds nothing else"
    assert len(queue) == len(set(queue))
    for i, n in enumerate(ns):
        if i in queue:
            assert nwg[i] == 1 and not rows[i]
            continue
        assert nwg[i] >= 2
        spans = sorted(rows[i])
        assert spans and spans[0][0] == 0 and spans[-1][1] == n
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 == b0
        assert sorted(ranks[i]) == list(range(nwg[i]))
        assert nwg[i] <= (n + 15) // 16
    # the queue is ordered by decreasing modelled cost: passes of tiles times
    # load round trips per pass (the planner's model, tpp=2, unroll=4, bw=64)
    def cost(n):
        passes = -(-(-(-n // 16)) // 2)
        return passes * (1 + -(-(-(-n // 64)) // 4)) + 1
    qc = [cost(int(ns[i])) for i in queue]
    assert qc == sorted(qc, reverse=True)


def test_planner_invariants(plan_exe):
    rng = np.random.default_rng(1403)
    cases = [([], 256), ([1], 256), ([4096], 256), ([17, 16, 15], 1), ([100000], 64),
             ([4096] * 3, 4), ([4096] * 3 + [256], 4), ([65536, 65536], 3),
             # equal systems at 1.5 workgroups each: shrinking one share to a
             # whole-system job must still leave room for it
             ([4096] * 4, 6), ([4096] * 8, 12), ([4096] * 40, 60), ([2048] * 341, 512)]
    for _ in range(40):
        count = int(rng.integers(1, 400))
        ns = np.exp(rng.uniform(np.log(1), np.log(20000), count)).astype(int) + 1
        cases.append((list(ns), int(rng.integers(1, 1024))))
    for ns, cap in cases:
        grid, nwg, wgs, queue = _plan(plan_exe, ns, cap)
        _check_plan(ns, cap, grid, nwg, wgs, queue)


def test_planner_on_the_batched_workload(plan_exe):
    """256 systems with n log-uniform in [256, 4096] on 512 resident
    workgroups: the largest systems are split, each share at least one full
    pass of tiles, and the rest wait in the queue, largest first."""
    rng = np.random.default_rng(7)
    ns = np.exp(rng.uniform(np.log(256), np.log(4096), 256)).astype(int)
    grid, nwg, wgs, queue = _plan(plan_exe, ns, 512)
    _check_plan(list(ns), 512, grid, nwg, wgs, queue)
    split = [i for i in range(len(ns)) if nwg[i] > 1]
    assert split and queue
    assert min(ns[i] for i in split) >= max(ns[i] for i in queue) // 2
    for g, jobs in wgs.items():
        for s, r, r0, r1 in jobs:
            assert r1 - r0 >= 32 or r1 == ns[s]


def _items(exe, ns, capacity, tpp=2, elem=4, groups=1):
    inp = (f"items {capacity} {tpp} {elem} {groups} {len(ns)} " +
           " ".join(str(int(v)) for v in ns))
    out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout
    grid, ranges, items, goff = 0, {}, [], []
    for ln in out.splitlines():
        p = ln.split()
        if p[0] == "grid":
            grid = int(p[1])
        elif p[0] == "goff":
            assert int(p[1]) == len(goff)
            goff.append(int(p[2]))
        elif p[0] == "range":
            ranges[int(p[1])] = (int(p[2]), int(p[3]))
        else:
            assert int(p[1]) == len(items)
            items.append(tuple(map(int, p[2:])))
    return grid, ranges, items, goff


def test_lockstep_items_invariants(plan_exe):
    """Work items of the lockstep schedule: each system's rows covered once,
    in order, by a contiguous item range inside one group; groups partition
    the items in order; chunks are whole passes of 16 * tpp rows except a
    system's last; systems by decreasing n within a group; the groups' bytes
    balanced as the largest-first greedy rule makes them; item sizes near the
    target; grid = min(capacity, items)."""
    rng = np.random.default_rng(5805)
    cases = [([], 512, 2, 4, 1), ([1], 512, 2, 4, 8), ([16384], 512, 2, 4, 8),
             ([32768], 256, 4, 2, 1), ([5, 0, 7], 8, 4, 4, 8), ([4096] * 3 + [256], 4, 2, 2, 8),
             ([4096] * 20, 256, 4, 4, 8)]
    for _ in range(30):
        count = int(rng.integers(1, 300))
        ns = np.exp(rng.uniform(np.log(1), np.log(20000), count)).astype(int)
        cases.append((list(ns), int(rng.integers(1, 1024)), int(rng.choice([2, 4])),
                      int(rng.choice([2, 4, 8])), int(rng.choice([1, 8]))))
    for ns, cap, tpp, elem, groups in cases:
        grid, ranges, items, goff = _items(plan_exe, ns, cap, tpp, elem, groups)
        assert len(goff) == groups + 1 and goff[0] == 0 and goff[-1] == len(items)
        assert all(a <= b for a, b in zip(goff, goff[1:]))
        group_of = {}
        for g in range(groups):
            for j in range(goff[g], goff[g + 1]):
                group_of[j] = g
        # greedy balance: each group's load <= lightest group's load + largest system
        loads = [0] * groups
        for s_, (a, b) in ranges.items():
            if b > a:
                g = group_of[a]
                assert all(group_of[j] == g for j in range(a, b))
                loads[g] += int(ns[s_]) ** 2
        if ns:
            assert max(loads) <= min(loads) + max(int(v) for v in ns) ** 2
        assert grid == min(max(1, cap), len(items))
        total = sum(int(v) * int(v) * elem for v in ns)
        target = min(2 << 20, max(128 << 10, total / (8 * max(1, cap))))
        seen = []
        for s_, (a, b) in ranges.items():
            n = int(ns[s_])
            assert (b > a) == (n > 0)
            rows = [items[j] for j in range(a, b)]
            assert all(it[0] == s_ for it in rows)
            r = 0
            for j, (_, r0, r1) in enumerate(rows):
                assert r0 == r and r1 > r0
                if j < len(rows) - 1:
                    assert (r1 - r0) % (16 * tpp) == 0
                    assert (r1 - r0 - 16 * tpp) * n * elem < target
                r = r1
            assert r == n
            seen.extend(range(a, b))
        assert sorted(seen) == list(range(len(items)))
        for g in range(groups):
            grp = items[goff[g]:goff[g + 1]]
            order = [it[0] for j, it in enumerate(grp) if j == 0 or grp[j - 1][0] != it[0]]
            assert [int(ns[i]) for i in order] == sorted((int(ns[i]) for i in order),
                                                         reverse=True)


# ---- serving arena -----------------------------------------------------------

def test_serving_arena_invariants(tmp_path):
    """Best-fit arena of the serving engine on random alloc/free sequences:
    aligned, disjoint blocks inside reserved slabs; the reservation limit is
    kept; a refusal only when no free block fits; freeing everything
    coalesces each slab back into one block and the space is reused; no slab
    outlives the arena."""
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "arena_check.cpp"),
                    os.path.join(PKG, "csrc", "arena.cpp"), "-o", str(exe)], check=True)
    for seed, ops, limit_mb, slab_mb in [(1, 20000, 4096, 1024), (2, 20000, 4096, 1024),
                                         (3, 5000, 64, 4096), (4, 20000, 1024, 16)]:
        out = subprocess.run([str(exe), str(seed), str(ops), str(limit_mb), str(slab_mb)],
                             capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
