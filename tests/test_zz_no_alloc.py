"""goat_sinkhorn_noalloc (the LOT solve without a workspace: its state in a
static device array) against goat_sinkhorn with a caller workspace, through
the C ABI: the same kernels on the same inputs give the same bits. Two calls
in a row, the second on a smaller problem, so the second reads nothing the
first left in the shared array; every start mode; the refusals."""
import ctypes

import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_VP, _I, _F, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    lib = goat.lib()
    lib.goat_sinkhorn_noalloc.restype = _I
    lib.goat_sinkhorn_noalloc.argtypes = [_I, _VP, _I, _VP, _F, _VP, _VP, _I, _VP, _I, _F, _VP, _I, _VP, _VP,
                                          _VP, _VP]
    lib.goat_sinkhorn_noalloc_max_n.restype = _I
    lib.goat_sinkhorn_noalloc_scratch_bytes.restype = _SZ
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _problem(n, seed):
    """G with rows padded to a multiple of 64 floats (the layout both entry
    points sweep without repacking)."""
    g = I.rho_er_pair(n, min(0.5, 12.0 / n), 0.9, seed)
    P = O.sinkhorn_knopp(I.uniform_matrix(n, seed + 1).astype(np.float64) + 0.05)
    G = O.gradient(g.A.astype(float), g.B.astype(float), 0.5 * (P + O.barycenter(n)))
    ld = (n + 63) // 64 * 64
    full = torch.zeros((n, ld), device="cuda")
    full[:, :n] = torch.as_tensor(G.astype(np.float32), device="cuda")
    return full[:, :n]


def _outputs(n):
    dev = "cuda"
    return dict(f=torch.full((n,), -7.0, device=dev), g=torch.full((n,), -7.0, device=dev),
                Q=torch.full((n, n), -7.0, device=dev), it=torch.full((1,), -7, dtype=torch.int32, device=dev),
                err=torch.full((1,), -7.0, device=dev), eps=torch.full((1,), -7.0, device=dev))


def _call(L, noalloc, G, init, max_iter, tol, g0=None, params=None):
    from paper_2111_05366_amd import goat
    n = G.shape[0]
    o = _outputs(n)
    if g0 is not None:
        o["g"].copy_(g0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    common = (n, _ptr(G), G.stride(0), None, _F(0.03), _ptr(o["f"]), _ptr(o["g"]), init, _ptr(params), max_iter,
              _F(tol), _ptr(o["Q"]), n, _ptr(o["it"]), _ptr(o["err"]), _ptr(o["eps"]))
    if noalloc:
        rc = L.goat_sinkhorn_noalloc(*common, stream)
    else:
        ws = goat.workspace(n, "fp32", True, G.device)
        rc = L.goat_sinkhorn(*common, _ptr(ws), ws.numel(), stream)
    torch.cuda.synchronize()
    assert rc == 0, L.goat_last_error()
    return o


def _same(a, b):
    for k in ("f", "g", "Q", "it", "err", "eps"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("init", [0, 1, 2])
def test_noalloc_equals_workspace_entry(L, init):
    from paper_2111_05366_amd import goat
    params = None
    if init == 2:
        from paper_2111_05366_amd import warmstart
        params = warmstart.load()
    # the larger problem first, then a smaller one in the same array
    for n, iters, tol in ((4500, 60, 1e-6), (1000, 25, 0.0)):
        print(f"noalloc init={init} n={n} iters={iters}", flush=True)
        G = _problem(n, 300 + n)
        g0 = torch.linspace(-0.5, 0.5, n, device="cuda") if init == 1 else None
        ref = _call(L, False, G, init, iters, tol, g0, params)
        got = _call(L, True, G, init, iters, tol, g0, params)
        _same(ref, got)
        print(f"  iters {int(got['it'].item())}, err {float(got['err'].item()):.2e}: identical")
    goat.release_workspace()


def test_noalloc_limits_and_refusals(L):
    nmax = L.goat_sinkhorn_noalloc_max_n()
    assert L.goat_sinkhorn_noalloc_scratch_bytes() == 64 << 20
    assert 10000 <= nmax < 20000
    dummy = ctypes.c_void_p(256)
    # above the largest size
    rc = L.goat_sinkhorn_noalloc(nmax + 1, dummy, nmax + 64, None, _F(0.03), None, None, 0, None, 10, _F(1e-6),
                                 None, nmax + 1, None, None, None, None)
    assert rc == -1 and b"goat_sinkhorn_noalloc_max_n" in L.goat_last_error()
    # a G the workspace entry would repack (rows not a multiple of 64 floats)
    n = 500
    G = torch.zeros((n, 500), device="cuda")
    rc = L.goat_sinkhorn_noalloc(n, _ptr(G), 500, None, _F(0.03), None, None, 0, None, 10, _F(1e-6), None, n,
                                 None, None, None, None)
    assert rc == -1 and b"repack" in L.goat_last_error()
    # with few sweeps it needs no repack and runs
    o = _outputs(n)
    Gp = _problem(n, 9).contiguous()
    rc = L.goat_sinkhorn_noalloc(n, _ptr(Gp), n, None, _F(0.03), _ptr(o["f"]), _ptr(o["g"]), 0, None, 4,
                                 _F(0.0), _ptr(o["Q"]), n, _ptr(o["it"]), _ptr(o["err"]), _ptr(o["eps"]), None)
    torch.cuda.synchronize()
    assert rc == 0 and int(o["it"].item()) == 4
