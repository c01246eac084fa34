"""Thin ctypes binding of libgoat (include/goat.h).

Argument marshalling only: every step of the GOAT path runs in the HIP
library. PyTorch supplies device memory (tensors' data pointers) and the
current HIP stream. Functions raise GoatError on a negative status and
RuntimeError if the library has not been built - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoat.so")

GOAT_OK, GOAT_EINVAL, GOAT_EHIP, GOAT_ENOMEM, GOAT_ENOTSUP = 0, -1, -2, -3, -4
PREC = {"fp32": 0, "bf16x2": 1, "bf16x3": 2, "fp8": 3}
INIT_COLD, INIT_G, INIT_MLP = 0, 1, 2


class GoatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"goat status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("eps_rel", ctypes.c_float), ("sk_tol", ctypes.c_float), ("sk_max", ctypes.c_int),
                ("fw_max", ctypes.c_int), ("fw_tol", ctypes.c_float), ("prec", ctypes.c_int),
                ("symmetric", ctypes.c_int), ("proj", ctypes.c_int), ("warm", ctypes.c_int),
                ("stop_on_stall", ctypes.c_int), ("check_every", ctypes.c_int),
                ("lap", ctypes.c_int), ("sk_g24", ctypes.c_int), ("reserved", ctypes.c_int * 3),
                ("mlp_params", ctypes.c_void_p)]


class IterRecord(ctypes.Structure):
    _fields_ = [("fP", ctypes.c_double), ("fQ", ctypes.c_double), ("c", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("t", ctypes.c_double),
                ("dist2", ctypes.c_double), ("eps", ctypes.c_float), ("sk_err", ctypes.c_float),
                ("sk_iters", ctypes.c_int), ("pad", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("fw_iters", ctypes.c_int), ("sk_iters_total", ctypes.c_int),
                ("sk_capped", ctypes.c_int), ("lap_device", ctypes.c_int),
                ("f_final", ctypes.c_double), ("score", ctypes.c_double),
                ("ms_loop", ctypes.c_double), ("ms_lap", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


class LapStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_longlong), ("rounds_launched", ctypes.c_longlong),
                ("tail_bids", ctypes.c_longlong), ("phases", ctypes.c_int), ("shift", ctypes.c_int), ("resolution_bits", ctypes.c_int),
                ("list_bids", ctypes.c_int), ("skipped_phases", ctypes.c_int)]


class Pair(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("ld", ctypes.c_int), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("U", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("problems", ctypes.c_int), ("fw_iters_total", ctypes.c_int),
                ("sk_iters_total", ctypes.c_longlong), ("sk_capped", ctypes.c_int),
                ("launches", ctypes.c_int), ("ms_graph", ctypes.c_double), ("ms_lap", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("lap_bids", ctypes.c_longlong)]


_lib = None
_VP, _I, _F, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t


def lib():
    """Load libgoat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_05366_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.goat_version.restype = _I
    L.goat_last_error.restype = ctypes.c_char_p
    L.goat_workspace_size.restype = _SZ
    L.goat_workspace_size.argtypes = [_I, _I, _I]
    L.goat_default_options.argtypes = [ctypes.POINTER(Options)]
    L.goat_grad.restype = _I
    L.goat_grad.argtypes = [_I, _VP, _VP, _I, _VP, _I, _VP, _I, _I, _I, _VP, _SZ, _VP]
    L.goat_pack.restype = _I
    L.goat_pack.argtypes = [_I, _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]
    L.goat_grad_packed.restype = _I
    L.goat_grad_packed.argtypes = [_I, _VP, _I, _VP, _I, _I, _I, _VP, _SZ, _VP]
    L.goat_sinkhorn.restype = _I
    L.goat_sinkhorn.argtypes = [_I, _VP, _I, _VP, _F, _VP, _VP, _I, _VP, _I, _F, _VP, _I, _VP, _VP, _VP,
                                _VP, _SZ, _VP]
    L.goat_linesearch.restype = _I
    L.goat_linesearch.argtypes = [_I, _VP, _VP, _VP, _VP, _I, _VP, _VP, _SZ, _VP]
    L.goat_solve.restype = _I
    L.goat_solve.argtypes = [_I, _VP, _VP, _I, _VP, ctypes.POINTER(Options), _VP,
                             ctypes.POINTER(Stats), ctypes.POINTER(IterRecord), _I, _VP, _VP, _SZ, _VP]
    L.goat_lap_max.restype = _I
    L.goat_lap_max.argtypes = [_I, _VP, _I, _VP]
    L.goat_score.restype = _I
    L.goat_score.argtypes = [_I, _VP, _VP, _I, _VP, _VP, _VP, _SZ, _VP]
    L.goat_lap_device_workspace_size.restype = _SZ
    L.goat_lap_device_workspace_size.argtypes = [_I]
    L.goat_lap_device_workspace_min.restype = _SZ
    L.goat_lap_device_workspace_min.argtypes = [_I]
    L.goat_lap_device.restype = _I
    L.goat_lap_device.argtypes = [_I, _VP, _I, _VP, _VP, _SZ, ctypes.c_longlong, ctypes.POINTER(LapStats), _VP]
    L.goat_nominate.restype = _I
    L.goat_nominate.argtypes = [_I, _I, _VP, _I, _I, _VP, _VP, _VP]
    L.goat_run_begin.restype = _I
    L.goat_run_begin.argtypes = [_I, _VP, _VP, _I, _VP, ctypes.POINTER(Options), _VP, _SZ, _VP,
                                 ctypes.POINTER(ctypes.c_void_p)]
    L.goat_run_steps.restype = _I
    L.goat_run_steps.argtypes = [_VP, _I, ctypes.POINTER(IterRecord), _I, ctypes.POINTER(ctypes.c_int)]
    L.goat_run_finish.restype = _I
    L.goat_run_finish.argtypes = [_VP, _VP, ctypes.POINTER(Stats), _VP, _I]
    L.goat_run_gradient.restype = _I
    L.goat_run_gradient.argtypes = [_VP, _VP, _I]
    L.goat_run_direction.restype = _I
    L.goat_run_direction.argtypes = [_VP, _VP, _I]
    L.goat_run_set_sinkhorn.restype = _I
    L.goat_run_set_sinkhorn.argtypes = [_VP, _I, _F]
    L.goat_run_free.restype = None
    L.goat_run_free.argtypes = [_VP]
    L.goat_mlp_param_count.restype = _I
    L.goat_mlp_workspace_size.restype = _SZ
    L.goat_mlp_workspace_size.argtypes = [_I]
    L.goat_mlp_features.restype = _I
    L.goat_mlp_features.argtypes = [_I, _VP, _I, _VP, _VP, _VP, _SZ, _VP]
    L.goat_mlp_forward.restype = _I
    L.goat_mlp_forward.argtypes = [_I, _VP, _VP, _VP, _VP]
    L.goat_mlp_backward.restype = _I
    L.goat_mlp_backward.argtypes = [_I, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]
    L.goat_mlp_adam.restype = _I
    L.goat_mlp_adam.argtypes = [_VP, _VP, _VP, _VP, _I, _F, _VP]
    L.goat_profile_enable.restype = _I
    L.goat_profile_enable.argtypes = [_I, _I]
    L.goat_profile_read.restype = _I
    L.goat_profile_read.argtypes = [_I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    L.goat_seeded_workspace_size.restype = _SZ
    L.goat_seeded_workspace_size.argtypes = [_I, _I, _I, _I, _I]
    L.goat_solve_seeded.restype = _I
    L.goat_solve_seeded.argtypes = [_I, _VP, _I, _I, _VP, _I, _I, _VP, _VP, _I, ctypes.POINTER(Options), _VP,
                                    ctypes.POINTER(Stats), ctypes.POINTER(IterRecord), _I, _VP, _SZ, _VP]
    L.goat_random_init_workspace_size.restype = _SZ
    L.goat_random_init_workspace_size.argtypes = [_I]
    L.goat_random_init.restype = _I
    L.goat_random_init.argtypes = [_I, _VP, _I, _VP, _I, _F, _I, _VP, _VP, _VP, _SZ, _VP]
    L.goat_solve_restarts_workspace_size.restype = _SZ
    L.goat_solve_restarts_workspace_size.argtypes = [_I, _I, _I, _I]
    L.goat_solve_restarts.restype = _I
    L.goat_solve_restarts.argtypes = [_I, _VP, _VP, _I, _VP, _I, _I, ctypes.POINTER(Options), _VP, _VP, _VP,
                                      ctypes.POINTER(Stats), _VP, _SZ, _VP]
    L.goat_batch_workspace_size.restype = _I
    L.goat_batch_workspace_size.argtypes = [ctypes.POINTER(Pair), _I, _I, ctypes.POINTER(Options),
                                            ctypes.POINTER(ctypes.c_size_t)]
    L.goat_batch_create.restype = _I
    L.goat_batch_create.argtypes = [ctypes.POINTER(Pair), _I, _I, ctypes.POINTER(Options), _VP, _SZ,
                                    ctypes.POINTER(ctypes.c_void_p)]
    L.goat_batch_launch.restype = _I
    L.goat_batch_launch.argtypes = [_VP, _VP]
    L.goat_batch_results.restype = _I
    L.goat_batch_results.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(IterRecord), _I, _VP,
                                     ctypes.POINTER(BatchStats)]
    L.goat_batch_get_P.restype = _I
    L.goat_batch_get_P.argtypes = [_VP, _I, _I, _VP, _I, _VP]
    L.goat_batch_destroy.restype = None
    L.goat_batch_destroy.argtypes = [_VP]
    L.goat_tune.restype = _I
    L.goat_tune.argtypes = [_I, _I, _VP]
    L.goat_tune_get.restype = _I
    L.goat_tune_get.argtypes = [_I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    _lib = L
    return L


def _check(status):
    if status != GOAT_OK:
        raise GoatError(status, lib().goat_last_error().decode())


def version() -> int:
    return lib().goat_version()


def workspace_size(n: int, prec: str = "fp32", symmetric: bool = True) -> int:
    return int(lib().goat_workspace_size(n, PREC[prec], int(symmetric)))


def default_options(**kw) -> Options:
    o = Options()
    lib().goat_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        if k == "mlp_params" and v is not None and not isinstance(v, int):
            v = v.data_ptr()
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# --------------------------------------------------------------- torch side

def _torch():
    import torch
    return torch


_ws_cache: dict = {}


def workspace(n: int, prec: str = "fp32", symmetric: bool = True, device=None):
    """A cached device workspace tensor sized for every call at (n, prec)."""
    torch = _torch()
    device = device or torch.device("cuda", torch.cuda.current_device())
    need = workspace_size(n, prec, symmetric)
    key = (str(device),)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need:
        _ws_cache.pop(key, None)
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def release_workspace():
    _ws_cache.clear()


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _mat(t, name):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name}: need a row-major float32 CUDA matrix")
    return t


def grad(A, B, P, prec: str = "fp32", symmetric: bool = True, out=None):
    """G = A P B^T + A^T P B on the device (goat_grad)."""
    torch = _torch()
    n = A.shape[0]
    for nm, t in (("A", A), ("B", B), ("P", P)):
        _mat(t, nm)
    if A.stride(0) != B.stride(0):
        raise ValueError("A and B must share a leading dimension")
    G = out if out is not None else torch.empty((n, n), dtype=torch.float32, device=A.device)
    ws = workspace(n, prec, symmetric, A.device)
    _check(lib().goat_grad(n, _ptr(A), _ptr(B), A.stride(0), _ptr(P), P.stride(0), _ptr(G), G.stride(0),
                           PREC[prec], int(symmetric), _ptr(ws), ws.numel(), _stream()))
    return G


class Packed:
    """A pair packed once into matrix-core operands (goat_pack), for many
    gradients by goat_grad_packed. Holds its own workspace; A and B may be
    released after construction."""

    def __init__(self, A, B, prec: str = "fp32", symmetric: bool = True):
        torch = _torch()
        _mat(A, "A"); _mat(B, "B")
        if A.stride(0) != B.stride(0):
            raise ValueError("A and B must share a leading dimension")
        self.n, self.prec, self.symmetric = A.shape[0], prec, bool(symmetric)
        need = workspace_size(self.n, prec, self.symmetric)
        self.ws = torch.empty(need, dtype=torch.uint8, device=A.device)
        _check(lib().goat_pack(self.n, _ptr(A), _ptr(B), A.stride(0), PREC[prec], int(self.symmetric),
                               _ptr(self.ws), need, _stream()))

    def grad(self, P, out=None):
        torch = _torch()
        _mat(P, "P")
        G = out if out is not None else torch.empty((self.n, self.n), dtype=torch.float32, device=P.device)
        _check(lib().goat_grad_packed(self.n, _ptr(P), P.stride(0), _ptr(G), G.stride(0), PREC[self.prec],
                                      int(self.symmetric), _ptr(self.ws), self.ws.numel(), _stream()))
        return G


@dataclass
class SinkhornOut:
    f: object
    g: object
    Q: object
    iters: object     # device int32[1]
    err: object       # device float32[1]
    eps: object       # device float32[1]


def sinkhorn(G, eps_rel: float = 0.03, max_iter: int = 1000, tol: float = 1e-6, g0=None, eps=None,
             want_Q: bool = True, mlp_params=None) -> SinkhornOut:
    """LOT direction on the device (goat_sinkhorn). Start: g0 if given, else
    the warm-start network if mlp_params is given, else cold."""
    torch = _torch()
    _mat(G, "G")
    n = G.shape[0]
    dev = G.device
    f = torch.empty(n, dtype=torch.float32, device=dev)
    g = torch.empty(n, dtype=torch.float32, device=dev) if g0 is None else g0.clone()
    Q = torch.empty((n, n), dtype=torch.float32, device=dev) if want_Q else None
    it = torch.zeros(1, dtype=torch.int32, device=dev)
    err = torch.zeros(1, dtype=torch.float32, device=dev)
    eps_out = torch.zeros(1, dtype=torch.float32, device=dev)
    eps_t = None
    if eps is not None:
        eps_t = torch.tensor([eps], dtype=torch.float32, device=dev)
    ws = workspace(n, "fp32", True, dev)
    init = INIT_G if g0 is not None else (INIT_MLP if mlp_params is not None else INIT_COLD)
    _check(lib().goat_sinkhorn(n, _ptr(G), G.stride(0), _ptr(eps_t), float(eps_rel), _ptr(f), _ptr(g),
                               init, _ptr(mlp_params), int(max_iter), float(tol),
                               _ptr(Q), Q.stride(0) if Q is not None else n, _ptr(it), _ptr(err),
                               _ptr(eps_out), _ptr(ws), ws.numel(), _stream()))
    return SinkhornOut(f, g, Q, it, err, eps_out)


def linesearch(P, Q, GP, GQ):
    """[fP, fQ, c, a, b, t, ||Q-P||^2, 0] as a device float64 tensor."""
    torch = _torch()
    n = P.shape[0]
    for nm, t in (("P", P), ("Q", Q), ("GP", GP), ("GQ", GQ)):
        _mat(t, nm)
    ld = P.stride(0)
    if not (Q.stride(0) == GP.stride(0) == GQ.stride(0) == ld):
        raise ValueError("P, Q, GP, GQ must share a leading dimension")
    out = torch.zeros(8, dtype=torch.float64, device=P.device)
    ws = workspace(n, "fp32", True, P.device)
    _check(lib().goat_linesearch(n, _ptr(P), _ptr(Q), _ptr(GP), _ptr(GQ), ld, _ptr(out), _ptr(ws),
                                 ws.numel(), _stream()))
    return out


def score(A, B, perm):
    """tr(A^T Pi B Pi^T) for a permutation (goat_score), float64 on device."""
    torch = _torch()
    n = A.shape[0]
    p = torch.as_tensor(np.asarray(perm, dtype=np.int32), device=A.device)
    out = torch.zeros(1, dtype=torch.float64, device=A.device)
    ws = workspace(n, "fp32", True, A.device)
    _check(lib().goat_score(n, _ptr(A), _ptr(B), A.stride(0), _ptr(p), _ptr(out), _ptr(ws), ws.numel(),
                            _stream()))
    return out


def lap_device(M, max_rounds: int = 0, precompute: bool = True):
    """Device assignment maximising sum_i M[i, perm i] on the quantised
    scores (goat_lap_device). M: row-major float32 device matrix.
    precompute=False passes the minimum workspace (scores converted in
    every scan; same result). Returns (perm int32 device tensor, LapStats)."""
    torch = _torch()
    _mat(M, "M")
    n = M.shape[0]
    if M.shape[1] != n:
        raise ValueError("M must be square")
    size = lib().goat_lap_device_workspace_size if precompute else lib().goat_lap_device_workspace_min
    ws = torch.empty(max(int(size(n)), 1), dtype=torch.uint8, device=M.device)
    perm = torch.empty(n, dtype=torch.int32, device=M.device)
    st = LapStats()
    _check(lib().goat_lap_device(n, _ptr(M), M.stride(0), _ptr(perm), _ptr(ws), ws.numel(), max_rounds,
                                 ctypes.byref(st), _stream()))
    return perm, st


NOMINATE_KMAX = 32


def nominate(P, k: int):
    """Soft matching (goat_nominate): for each row of the device float matrix
    P, the k columns with the largest scores, best first (ties by increasing
    column). Returns (idx int32 [rows, k], val float32 [rows, k]) on P's
    device."""
    torch = _torch()
    P = _mat(P, "P")
    rows, cols = P.shape
    idx = torch.empty((rows, k), dtype=torch.int32, device=P.device)
    val = torch.empty((rows, k), dtype=torch.float32, device=P.device)
    _check(lib().goat_nominate(rows, cols, _ptr(P), P.stride(0), k, _ptr(idx), _ptr(val), _stream()))
    return idx, val


def lap_max(M: np.ndarray) -> np.ndarray:
    """Host linear assignment maximising sum_i M[i, perm[i]] (goat_lap_max)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = M.shape[0]
    perm = np.empty(n, dtype=np.int32)
    _check(lib().goat_lap_max(n, M.ctypes.data_as(ctypes.c_void_p), n, perm.ctypes.data_as(ctypes.c_void_p)))
    return perm


@dataclass
class SolveResult:
    perm: np.ndarray
    stats: Stats
    history: list
    P: object


def solve(A, B, P0=None, return_P: bool = False, **opts) -> SolveResult:
    """Full GOAT for one pair (goat_solve). Options as in goat_options."""
    torch = _torch()
    _mat(A, "A"); _mat(B, "B")
    n = A.shape[0]
    if A.stride(0) != B.stride(0):
        raise ValueError("A and B must share a leading dimension")
    o = default_options(**opts)
    prec = {v: k for k, v in PREC.items()}[o.prec]
    ws = workspace(n, prec, bool(o.symmetric), A.device)
    perm = np.empty(n, dtype=np.int32)
    st = Stats()
    cap = max(o.fw_max, 1)
    hist = (IterRecord * cap)()
    Pout = torch.empty((n, n), dtype=torch.float32, device=A.device) if return_P else None
    if P0 is not None:
        _mat(P0, "P0")
        if P0.stride(0) != A.stride(0):
            raise ValueError("P0 must share A's leading dimension")
    _check(lib().goat_solve(n, _ptr(A), _ptr(B), A.stride(0), _ptr(P0), ctypes.byref(o),
                            perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st), hist, cap,
                            _ptr(Pout), _ptr(ws), ws.numel(), _stream()))
    h = []
    for k in range(st.fw_iters):
        r = hist[k]
        h.append(dict(fP=r.fP, fQ=r.fQ, c=r.c, a=r.a, b=r.b, t=r.t, dist2=r.dist2, eps=r.eps,
                      sk_err=r.sk_err, sk_iters=r.sk_iters))
    return SolveResult(perm.astype(np.int64), st, h, Pout)


def _records(hist, k):
    out = []
    for i in range(k):
        r = hist[i]
        out.append(dict(fP=r.fP, fQ=r.fQ, c=r.c, a=r.a, b=r.b, t=r.t, dist2=r.dist2, eps=r.eps,
                        sk_err=r.sk_err, sk_iters=r.sk_iters))
    return out


class Run:
    """Stepwise GOAT (goat_run_begin / steps / finish). A, B and the
    workspace stay referenced for the run's lifetime."""

    def __init__(self, A, B, P0=None, **opts):
        torch = _torch()
        _mat(A, "A"); _mat(B, "B")
        self.n = A.shape[0]
        self.A, self.B, self.P0 = A, B, P0
        self.opt = default_options(**opts)
        prec = {v: k for k, v in PREC.items()}[self.opt.prec]
        self.ws = torch.empty(workspace_size(self.n, prec, bool(self.opt.symmetric)), dtype=torch.uint8,
                              device=A.device)
        h = ctypes.c_void_p()
        _check(lib().goat_run_begin(self.n, _ptr(A), _ptr(B), A.stride(0), _ptr(P0), ctypes.byref(self.opt),
                                    _ptr(self.ws), self.ws.numel(), _stream(), ctypes.byref(h)))
        self.h = h
        self.history = []

    def steps(self, k: int) -> int:
        hist = (IterRecord * max(k, 1))()
        done = ctypes.c_int(0)
        _check(lib().goat_run_steps(self.h, k, hist, k, ctypes.byref(done)))
        self.history += _records(hist, done.value)
        return done.value

    def gradient(self):
        """Current grad f(P) of the run as an n x n device tensor."""
        torch = _torch()
        G = torch.empty((self.n, self.n), dtype=torch.float32, device=self.A.device)
        _check(lib().goat_run_gradient(self.h, _ptr(G), self.n))
        return G

    def direction(self):
        """The last iteration's Sinkhorn direction Q as an n x n device tensor."""
        torch = _torch()
        Q = torch.empty((self.n, self.n), dtype=torch.float32, device=self.A.device)
        _check(lib().goat_run_direction(self.h, _ptr(Q), self.n))
        return Q

    def set_sinkhorn(self, sk_max: int, sk_tol: float):
        """Sinkhorn cap and tolerance for the following steps."""
        _check(lib().goat_run_set_sinkhorn(self.h, int(sk_max), float(sk_tol)))

    def finish(self, return_P: bool = False):
        torch = _torch()
        perm = np.empty(self.n, dtype=np.int32)
        st = Stats()
        Pout = torch.empty((self.n, self.n), dtype=torch.float32, device=self.A.device) if return_P else None
        _check(lib().goat_run_finish(self.h, perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st), _ptr(Pout),
                                     self.n))
        return SolveResult(perm.astype(np.int64), st, list(self.history), Pout)

    def close(self):
        if self.h:
            lib().goat_run_free(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROF_SINKHORN_ROW, PROF_GEMM = 0, 1


def profile_enable(which: int, stride: int):
    _check(lib().goat_profile_enable(int(which), int(stride)))


def profile_read(which: int):
    """(summed ms, number of sampled launches) since the last read."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_longlong(0)
    _check(lib().goat_profile_read(int(which), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


# ------------------------------------------------------------ warm start

def mlp_param_count() -> int:
    return lib().goat_mlp_param_count()


def mlp_features(G, eps_dev):
    """Centred per-column features [n, 4] of G / eps (goat_mlp_features)."""
    torch = _torch()
    _mat(G, "G")
    n = G.shape[0]
    F = torch.empty((n, 4), dtype=torch.float32, device=G.device)
    ws = workspace(n, "fp32", True, G.device)
    _check(lib().goat_mlp_features(n, _ptr(G), G.stride(0), _ptr(eps_dev), _ptr(F), _ptr(ws), ws.numel(), _stream()))
    return F


def mlp_forward(F, params):
    torch = _torch()
    N = F.shape[0]
    y = torch.empty(N, dtype=torch.float32, device=F.device)
    _check(lib().goat_mlp_forward(N, _ptr(F), _ptr(params), _ptr(y), _stream()))
    return y


def mlp_backward(F, target, params, grad=None, loss=None, ws=None):
    """(grad [P], loss [1]) of the mean squared error (goat_mlp_backward)."""
    torch = _torch()
    N = F.shape[0]
    grad = grad if grad is not None else torch.empty_like(params)
    loss = loss if loss is not None else torch.zeros(1, dtype=torch.float32, device=F.device)
    need = int(lib().goat_mlp_workspace_size(N))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=F.device)
    _check(lib().goat_mlp_backward(N, _ptr(F), _ptr(target), _ptr(params), _ptr(grad), _ptr(loss), _ptr(ws),
                                   ws.numel(), _stream()))
    return grad, loss


def mlp_adam(grad, params, m, v, step: int, lr: float):
    _check(lib().goat_mlp_adam(_ptr(grad), _ptr(params), _ptr(m), _ptr(v), int(step), float(lr), _stream()))


# ------------------------------------------------------------ random starts, batches

def random_init(U, tol: float = 1e-6, max_iter: int = 1000):
    """P0 = (J + SK(U)) / 2 on the device (goat_random_init): (P, iters, err)."""
    torch = _torch()
    _mat(U, "U")
    n = U.shape[0]
    P = torch.empty((n, n), dtype=torch.float32, device=U.device)
    it = torch.zeros(1, dtype=torch.int32, device=U.device)
    err = torch.zeros(1, dtype=torch.float32, device=U.device)
    need = int(lib().goat_random_init_workspace_size(n))
    ws = torch.empty(need, dtype=torch.uint8, device=U.device) if need else None
    _check(lib().goat_random_init(n, _ptr(U), U.stride(0), _ptr(P), P.stride(0), float(tol), int(max_iter),
                                  _ptr(it), _ptr(err), _ptr(ws), need, _stream()))
    return P, it, err


@dataclass
class RestartsResult:
    perm: np.ndarray
    stats: Stats
    scores: np.ndarray
    best: int


def solve_restarts(A, B, U, restarts: int, **opts) -> RestartsResult:
    """GOAT from `restarts` random starts (goat_solve_restarts): U holds the
    starts' n x n positive draws stacked as a (restarts * n, n) tensor."""
    torch = _torch()
    _mat(A, "A"); _mat(B, "B"); _mat(U, "U")
    n = A.shape[0]
    if A.stride(0) != B.stride(0):
        raise ValueError("A and B must share a leading dimension")
    if U.shape[0] < restarts * n or U.shape[1] < n:
        raise ValueError("U must hold restarts stacked n x n matrices")
    o = default_options(**opts)
    need = int(lib().goat_solve_restarts_workspace_size(n, A.stride(0), o.prec, o.symmetric))
    ws = torch.empty(need, dtype=torch.uint8, device=A.device)
    perm = np.empty(n, dtype=np.int32)
    scores = np.empty(restarts, dtype=np.float64)
    best = ctypes.c_int(-1)
    st = Stats()
    _check(lib().goat_solve_restarts(n, _ptr(A), _ptr(B), A.stride(0), _ptr(U), U.stride(0), int(restarts),
                                     ctypes.byref(o), perm.ctypes.data_as(ctypes.c_void_p),
                                     scores.ctypes.data_as(ctypes.c_void_p), ctypes.byref(best),
                                     ctypes.byref(st), _ptr(ws), need, _stream()))
    return RestartsResult(perm.astype(np.int64), st, scores, best.value)


class Batch:
    """Many pairs x starts in one graph launch (goat_batch_*). `pairs` is a
    list of (A, B) or (A, B, U) device tensors; U holds `restarts` stacked
    n x n positive draws (restart r at rows r*n .. r*n+n-1) or is None.
    Tensors stay referenced for the batch's lifetime."""

    def __init__(self, pairs, restarts: int = 1, **opts):
        torch = _torch()
        self.keep = []
        arr = (Pair * len(pairs))()
        for k, pr in enumerate(pairs):
            A, B = pr[0], pr[1]
            U = pr[2] if len(pr) > 2 else None
            _mat(A, "A"); _mat(B, "B")
            if A.stride(0) != B.stride(0):
                raise ValueError("A and B of a pair must share a leading dimension")
            n = A.shape[0]
            if U is not None:
                if U.dtype != torch.float32 or not U.is_contiguous() or U.shape != (restarts * n, n) \
                        or A.stride(0) != n:
                    raise ValueError("U must be a contiguous float32 (restarts*n, n) tensor and ld == n")
            arr[k] = Pair(n, A.stride(0), _ptr(A), _ptr(B), _ptr(U))
            self.keep += [A, B, U]
        self.pairs = arr
        self.npairs = len(pairs)
        self.restarts = restarts
        self.n = [p.n for p in arr]
        self.opt = default_options(**opts)
        need = ctypes.c_size_t(0)
        _check(lib().goat_batch_workspace_size(arr, len(pairs), restarts, ctypes.byref(self.opt),
                                               ctypes.byref(need)))
        self.ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=pairs[0][0].device)
        h = ctypes.c_void_p()
        _check(lib().goat_batch_create(arr, len(pairs), restarts, ctypes.byref(self.opt), _ptr(self.ws),
                                       self.ws.numel(), ctypes.byref(h)))
        self.h = h

    def launch(self):
        _check(lib().goat_batch_launch(self.h, _stream()))

    def results(self, hist_cap: int | None = None):
        cap = hist_cap or self.opt.fw_max
        N = self.npairs * self.restarts
        perm = np.empty(sum(self.n), dtype=np.int32)
        score = np.empty(self.npairs, dtype=np.float64)
        best = np.empty(self.npairs, dtype=np.int32)
        allsc = np.empty(N, dtype=np.float64)
        hist = (IterRecord * (N * cap))()
        fwd = np.empty(N, dtype=np.int32)
        st = BatchStats()
        _check(lib().goat_batch_results(self.h, perm.ctypes.data_as(ctypes.c_void_p),
                                        score.ctypes.data_as(ctypes.c_void_p), best.ctypes.data_as(ctypes.c_void_p),
                                        allsc.ctypes.data_as(ctypes.c_void_p), hist, cap,
                                        fwd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)))
        perms, o = [], 0
        for n in self.n:
            perms.append(perm[o:o + n].astype(np.int64))
            o += n
        histories = []
        for k in range(N):
            recs = [hist[k * cap + f] for f in range(min(int(fwd[k]), cap))]
            histories.append([dict(fP=r.fP, fQ=r.fQ, c=r.c, a=r.a, b=r.b, t=r.t, dist2=r.dist2, eps=r.eps,
                                   sk_err=r.sk_err, sk_iters=r.sk_iters) for r in recs])
        return dict(perm=perms, score=score, best=best, all_scores=allsc.reshape(self.npairs, self.restarts),
                    history=histories, fw_iters=fwd.reshape(self.npairs, self.restarts), stats=st)

    def get_P(self, pair: int, restart: int = 0):
        torch = _torch()
        n = self.n[pair]
        P = torch.empty((n, n), dtype=torch.float32, device=self.ws.device)
        _check(lib().goat_batch_get_P(self.h, pair, restart, _ptr(P), n, _stream()))
        return P

    def close(self):
        if getattr(self, "h", None):
            lib().goat_batch_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(pairs, restarts: int = 1, **opts):
    b = Batch(pairs, restarts, **opts)
    try:
        b.launch()
        return b.results()
    finally:
        b.close()


def tune(n_max: int, reps: int = 3):
    _check(lib().goat_tune(int(n_max), int(reps), _stream()))


def tune_get(n: int):
    L = ctypes.c_int(0)
    w = ctypes.c_int(0)
    _check(lib().goat_tune_get(int(n), ctypes.byref(L), ctypes.byref(w)))
    return L.value, w.value


def solve_seeded(A, B, seeds_A=(), seeds_B=(), pad: str = "naive", **opts) -> SolveResult:
    """Seeded / unequal-size GOAT (goat_solve_seeded). perm[i] is the B
    vertex matched to A vertex i, -1 for a dummy."""
    torch = _torch()
    _mat(A, "A"); _mat(B, "B")
    nA, nB = A.shape[0], B.shape[0]
    sA = np.ascontiguousarray(np.asarray(seeds_A, dtype=np.int32))
    sB = np.ascontiguousarray(np.asarray(seeds_B, dtype=np.int32))
    if sA.shape != sB.shape:
        raise ValueError("seeds_A and seeds_B must have the same length")
    m = int(sA.shape[0])
    o = default_options(**opts)
    need = int(lib().goat_seeded_workspace_size(nA, nB, m, o.prec, o.symmetric))
    if need == 0:
        raise ValueError("bad sizes, seed count or precision")
    ws = torch.empty(need, dtype=torch.uint8, device=A.device)
    perm = np.empty(nA, dtype=np.int32)
    st = Stats()
    cap = max(o.fw_max, 1)
    hist = (IterRecord * cap)()
    _check(lib().goat_solve_seeded(nA, _ptr(A), A.stride(0), nB, _ptr(B), B.stride(0), m,
                                   sA.ctypes.data_as(ctypes.c_void_p) if m else None,
                                   sB.ctypes.data_as(ctypes.c_void_p) if m else None,
                                   {"naive": 0, "adopted": 1}[pad], ctypes.byref(o),
                                   perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st), hist, cap,
                                   _ptr(ws), ws.numel(), _stream()))
    return SolveResult(perm.astype(np.int64), st, _records(hist, st.fw_iters), None)
