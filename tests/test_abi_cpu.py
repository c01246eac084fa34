"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/goat.h declares, rejects bad arguments before touching the device,
and its host linear assignment matches brute force and SciPy."""
import ctypes
import itertools
import os
import re
import subprocess

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "goat.h")


def _ensure_built():
    from paper_2111_05366_amd import goat
    if not os.path.exists(goat.LIB_PATH):
        from paper_2111_05366_amd import build
        build.build()
    return goat


@pytest.fixture(scope="module")
def G():
    return _ensure_built()


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(goat_\w+)\s*\(", txt)))


def test_exports_every_declared_symbol(G):
    names = _declared()
    assert {"goat_grad", "goat_sinkhorn", "goat_linesearch", "goat_solve"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (goat_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = G.lib()
    for n in names:
        assert hasattr(L, n)


def test_version_and_sizes(G):
    assert G.version() >= 100
    s1 = G.workspace_size(64, "fp32", True)
    s2 = G.workspace_size(64, "fp32", False)
    s3 = G.workspace_size(1000, "bf16x3", True)
    assert 0 < s1 < s2 and s3 > s1
    assert G.lib().goat_workspace_size(0, 0, 1) == 0
    assert G.lib().goat_workspace_size(10, 7, 1) == 0


def test_options_defaults(G):
    o = G.default_options()
    assert abs(o.eps_rel - 0.03) < 1e-7 and abs(o.sk_tol - 1e-6) < 1e-12
    assert o.sk_max == 1000 and o.fw_max == 30 and o.prec == 0 and o.symmetric == 1
    assert o.stop_on_stall == 1


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_host_lap_brute_force(G, n):
    rng = np.random.default_rng(200 + n)
    for _ in range(6):
        M = rng.normal(size=(n, n))
        best = max(sum(M[i, p[i]] for i in range(n)) for p in itertools.permutations(range(n)))
        perm = G.lap_max(M)
        assert sorted(perm) == list(range(n))
        assert M[np.arange(n), perm].sum() == pytest.approx(best, abs=1e-12)


@pytest.mark.parametrize("n", [50, 300, 1000])
def test_host_lap_vs_scipy(G, n):
    rng = np.random.default_rng(300 + n)
    M = rng.random((n, n))
    perm = G.lap_max(M)
    r, c = linear_sum_assignment(M, maximize=True)
    assert M[np.arange(n), perm].sum() == pytest.approx(M[r, c].sum(), abs=1e-9)
    # integer costs: many ties, value still optimal
    Mi = rng.integers(0, 5, size=(n, n)).astype(float)
    perm = G.lap_max(Mi)
    r, c = linear_sum_assignment(Mi, maximize=True)
    assert Mi[np.arange(n), perm].sum() == Mi[r, c].sum()


def test_host_lap_tie_example(G):
    from conftest import load_golden
    d = load_golden("tie_example.txt")
    M = np.array(d["M"])
    assert M[np.arange(4), G.lap_max(M)].sum() == 183
    assert M[np.arange(4), G.lap_max(-M)].sum() == 172
    p = G.lap_max(np.zeros((6, 6)))
    assert sorted(p) == list(range(6))


def test_host_lap_smooth_plan_fast(G):
    """A smooth entropic-looking plan (the typical final P) at n=2000."""
    import time
    n = 2000
    rng = np.random.default_rng(8)
    S = rng.normal(size=(n, 8)) @ rng.normal(size=(8, n)) + 0.3 * rng.normal(size=(n, n))
    M = np.exp(S / 0.5)
    M /= M.sum(1, keepdims=True)
    t = time.time()
    perm = G.lap_max(M)
    dt = time.time() - t
    r, c = linear_sum_assignment(M, maximize=True)
    assert M[np.arange(n), perm].sum() == pytest.approx(M[r, c].sum(), rel=1e-12)
    assert dt < 10.0


def test_host_lap_near_permutation_fast(G):
    import time
    n = 3000
    rng = np.random.default_rng(7)
    pi = rng.permutation(n)
    M = 0.01 * rng.random((n, n))
    M[np.arange(n), pi] += 1.0
    t = time.time()
    perm = G.lap_max(M)
    assert (perm == pi).all()
    assert time.time() - t < 5.0


def test_host_lap_rejects_nonfinite(G):
    M = np.ones((3, 3)); M[1, 1] = np.nan
    with pytest.raises(G.GoatError) as e:
        G.lap_max(M)
    assert e.value.status == G.GOAT_EINVAL


def test_bad_arguments_rejected_before_device(G):
    L = G.lib()
    s = L.goat_grad(0, None, None, 0, None, 0, None, 0, 0, 1, None, 0, None)
    assert s == G.GOAT_EINVAL
    assert b"n < 1" in L.goat_last_error()
    s = L.goat_grad(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 2, ctypes.c_void_p(16), 4,
                    ctypes.c_void_p(16), 4, 0, 1, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # ld < n
    s = L.goat_grad(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4,
                    ctypes.c_void_p(16), 4, 9, 1, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # unknown precision
    s = L.goat_grad(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4,
                    ctypes.c_void_p(16), 4, 0, 1, ctypes.c_void_p(16), 16, None)
    assert s == G.GOAT_ENOMEM          # workspace too small
    s = L.goat_sinkhorn(4, ctypes.c_void_p(16), 4, None, ctypes.c_float(0.0), None, None, 0, None, 10,
                        ctypes.c_float(1e-6), None, 4, None, None, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # eps_rel <= 0
    s = L.goat_sinkhorn(4, ctypes.c_void_p(16), 4, None, ctypes.c_float(0.03), None, None, 1, None, 10,
                        ctypes.c_float(1e-6), None, 4, None, None, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # warm start without g
    s = L.goat_sinkhorn(4, ctypes.c_void_p(16), 4, None, ctypes.c_float(0.03), None, None, 2, None, 10,
                        ctypes.c_float(1e-6), None, 4, None, None, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # network start without parameters
    assert b"GOAT_INIT_MLP needs mlp_params" in L.goat_last_error()
    s = L.goat_sinkhorn(30000, ctypes.c_void_p(16), 30000, None, ctypes.c_float(0.03), None, None, 2,
                        ctypes.c_void_p(16), 10, ctypes.c_float(1e-6), None, 30000, None, None, None,
                        ctypes.c_void_p(16), 1 << 40, None)
    assert s == G.GOAT_EINVAL          # the network's size limit
    s = L.goat_sinkhorn(4, ctypes.c_void_p(16), 4, None, ctypes.c_float(0.03), None, None, 3, None, 10,
                        ctypes.c_float(1e-6), None, 4, None, None, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # unknown start
    s = L.goat_sinkhorn(4, ctypes.c_void_p(16), 4, None, ctypes.c_float(0.03), None, None, 0, None, 10,
                        ctypes.c_float(float("nan")), None, 4, None, None, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL          # non-finite tol
    dummy = ctypes.c_void_p(16)
    assert L.goat_pack(0, dummy, dummy, 4, 0, 1, dummy, 1 << 30, None) == G.GOAT_EINVAL
    assert L.goat_pack(4, dummy, None, 4, 0, 1, dummy, 1 << 30, None) == G.GOAT_EINVAL
    assert L.goat_pack(4, dummy, dummy, 4, 7, 1, dummy, 1 << 30, None) == G.GOAT_EINVAL
    assert L.goat_pack(4, dummy, dummy, 4, 0, 1, dummy, 16, None) == G.GOAT_ENOMEM
    assert L.goat_grad_packed(4, dummy, 3, dummy, 4, 0, 1, dummy, 1 << 30, None) == G.GOAT_EINVAL
    assert L.goat_grad_packed(4, dummy, 4, dummy, 4, 1, 1, dummy, 16, None) == G.GOAT_ENOMEM
    s = L.goat_linesearch(4, None, None, None, None, 4, None, None, 0, None)
    assert s == G.GOAT_EINVAL
    o = G.default_options(sk_max=0)
    s = L.goat_solve(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, None, ctypes.byref(o),
                     ctypes.c_void_p(16), None, None, 0, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL
    o = G.default_options(sk_g24=1)            # the 24-bit copy needs a mixed precision
    s = L.goat_solve(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, None, ctypes.byref(o),
                     ctypes.c_void_p(16), None, None, 0, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL and b"sk_g24" in L.goat_last_error()
    o = G.default_options(sk_g24=2, prec="bf16x2")
    s = L.goat_solve(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, None, ctypes.byref(o),
                     ctypes.c_void_p(16), None, None, 0, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL
    # the mixed forms' workspace holds the 24-bit copy (3 n_p^2 bytes more than fp32's operands need)
    assert L.goat_workspace_size(1000, 1, 1) >= 3 * 1024 * 1024
    o = G.default_options(eps_rel=float("inf"))
    s = L.goat_solve(4, ctypes.c_void_p(16), ctypes.c_void_p(16), 4, None, ctypes.byref(o),
                     ctypes.c_void_p(16), None, None, 0, None, ctypes.c_void_p(16), 1 << 30, None)
    assert s == G.GOAT_EINVAL


def test_batch_arguments_rejected_before_device(G):
    L = G.lib()
    pairs = (G.Pair * 2)(G.Pair(50, 50, 16, 32, None), G.Pair(400, 400, 48, 64, None))
    need = ctypes.c_size_t(0)
    o = G.default_options()
    assert L.goat_batch_workspace_size(pairs, 2, 8, ctypes.byref(o), ctypes.byref(need)) == G.GOAT_OK
    # 16 problems: at least P, Q, G_P, G_Q, T per problem and A, B per pair
    np_ = [64, 416]
    assert need.value >= sum(8 * 5 * 4 * m * m + 2 * 4 * m * m for m in np_)
    h = ctypes.c_void_p()
    assert L.goat_batch_create(pairs, 2, 8, ctypes.byref(o), ctypes.c_void_p(256), 1024,
                               ctypes.byref(h)) == G.GOAT_ENOMEM
    assert L.goat_batch_workspace_size(pairs, 2, 0, ctypes.byref(o), ctypes.byref(need)) == G.GOAT_EINVAL
    for bad in (G.Pair(0, 4, 16, 32, None), G.Pair(1025, 1025, 16, 32, None), G.Pair(8, 4, 16, 32, None),
                G.Pair(8, 8, None, 32, None)):
        one = (G.Pair * 1)(bad)
        assert L.goat_batch_workspace_size(one, 1, 1, ctypes.byref(o), ctypes.byref(need)) == G.GOAT_EINVAL
    for kw, status in ((dict(prec=G.PREC["bf16x3"]), G.GOAT_ENOTSUP), (dict(warm=2), G.GOAT_ENOTSUP),
                       (dict(sk_max=0), G.GOAT_EINVAL), (dict(fw_max=0), G.GOAT_EINVAL),
                       (dict(eps_rel=float("nan")), G.GOAT_EINVAL), (dict(proj=2), G.GOAT_EINVAL),
                       (dict(sk_g24=1), G.GOAT_ENOTSUP)):
        ob = G.default_options(**kw)
        assert L.goat_batch_workspace_size(pairs, 2, 8, ctypes.byref(ob), ctypes.byref(need)) == status, kw
    assert L.goat_random_init(0, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4, ctypes.c_float(1e-6), 10,
                              None, None, None, 0, None) == G.GOAT_EINVAL
    assert L.goat_random_init(4, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4, ctypes.c_float(1e-6), 0,
                              None, None, None, 0, None) == G.GOAT_EINVAL
    assert L.goat_random_init(4, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4, ctypes.c_float(float("inf")),
                              10, None, None, None, 0, None) == G.GOAT_EINVAL
    # no workspace needed up to 1024 nodes; above, a short workspace is refused
    assert L.goat_random_init_workspace_size(1024) == 0
    need = L.goat_random_init_workspace_size(1025)
    assert need >= 4 * 1025 * 1025
    assert L.goat_random_init(1025, ctypes.c_void_p(16), 1025, ctypes.c_void_p(16), 1025, ctypes.c_float(1e-6),
                              10, None, None, ctypes.c_void_p(16), need - 1, None) == G.GOAT_ENOMEM
    assert b"goat_random_init_workspace_size" in L.goat_last_error()
    # restarts: sizes, pointers, count and workspace checked before the device
    o = G.default_options()
    ws_need = L.goat_solve_restarts_workspace_size(2000, 2000, 0, 1)
    assert ws_need >= L.goat_workspace_size(2000, 0, 1) + 4 * 2000 * 2000 + L.goat_random_init_workspace_size(2000)
    dummy = ctypes.c_void_p(16)
    for args, status in (((2000, dummy, dummy, 2000, dummy, 2000, 0), G.GOAT_EINVAL),
                         ((2000, dummy, dummy, 1999, dummy, 2000, 2), G.GOAT_EINVAL),
                         ((2000, None, dummy, 2000, dummy, 2000, 2), G.GOAT_EINVAL)):
        assert L.goat_solve_restarts(*args, ctypes.byref(o), dummy, None, None, None, dummy, ws_need,
                                     None) == status, args
    assert L.goat_solve_restarts(2000, dummy, dummy, 2000, dummy, 2000, 2, ctypes.byref(o), dummy, None, None,
                                 None, dummy, ws_need - 1, None) == G.GOAT_ENOMEM
    assert L.goat_tune(0, 1, None) == G.GOAT_EINVAL
    assert L.goat_tune_get(2000, None, None) == G.GOAT_EINVAL


def test_nominate_arguments_rejected_before_device(G):
    L = G.lib()
    dummy = ctypes.c_void_p(16)
    assert L.goat_nominate(0, 5, dummy, 5, 1, dummy, None, None) == G.GOAT_EINVAL      # rows < 1
    assert L.goat_nominate(4, 5, dummy, 5, 6, dummy, None, None) == G.GOAT_EINVAL      # k > cols
    assert L.goat_nominate(4, 50, dummy, 50, 33, dummy, None, None) == G.GOAT_EINVAL   # k > kmax
    assert L.goat_nominate(4, 5, dummy, 5, 0, dummy, None, None) == G.GOAT_EINVAL      # k < 1
    assert L.goat_nominate(4, 5, dummy, 4, 2, dummy, None, None) == G.GOAT_EINVAL      # ld < cols
    assert L.goat_nominate(4, 5, None, 5, 2, dummy, None, None) == G.GOAT_EINVAL       # null P
    assert G.NOMINATE_KMAX == 32


def test_lap_device_arguments_rejected_before_device(G):
    L = G.lib()
    dummy = ctypes.c_void_p(16)
    assert L.goat_lap_device_workspace_size(0) == 0
    assert L.goat_lap_device_workspace_size(1000) >= 1000 * (3 * 8 + 5 * 4)
    assert L.goat_lap_device(0, dummy, 1, dummy, dummy, 1 << 20, 0, None, None) == G.GOAT_EINVAL      # n < 1
    assert L.goat_lap_device(8, dummy, 7, dummy, dummy, 1 << 20, 0, None, None) == G.GOAT_EINVAL      # ld < n
    assert L.goat_lap_device(8, None, 8, dummy, dummy, 1 << 20, 0, None, None) == G.GOAT_EINVAL       # null M
    assert L.goat_lap_device(8, dummy, 8, None, dummy, 1 << 20, 0, None, None) == G.GOAT_EINVAL       # null perm
    assert L.goat_lap_device(1 << 20, dummy, 1 << 20, dummy, dummy, 1 << 40, 0, None, None) == G.GOAT_EINVAL  # n too large
    o = G.default_options(lap=2)
    s = L.goat_solve(4, dummy, dummy, 4, None, ctypes.byref(o), dummy, None, None, 0, None, dummy, 1 << 30, None)
    assert s == G.GOAT_EINVAL and b"assignment mode" in L.goat_last_error()


def test_ctypes_structs_match_header(tmp_path):
    """Every struct the binding mirrors has the size and field offsets of
    its declaration in goat.h (a mismatch lets the library write past a
    Python-side buffer). Checked by compiling the header with the host C
    compiler."""
    import os
    import shutil
    import subprocess
    from paper_2111_05366_amd import goat as G
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"goat_options": G.Options, "goat_iter_record": G.IterRecord, "goat_stats": G.Stats,
               "goat_lap_stats": G.LapStats, "goat_pair": G.Pair, "goat_batch_stats": G.BatchStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "goat.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I" + os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
