"""Plain FP64 CPU oracle for the GOAT hot path (graph matching via optimal
transport, arXiv 2111.05366).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module: only the tests, the smoke entry point and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library
(no kernels, headers, helpers, tables or pre/post-processing).

Every function is written for a reader to check against the paper by eye:
float64 throughout, numpy matmul as the only library primitive for products,
no blocking, fusion or reordering beyond what the definitions state.

Conventions (readings of points the paper leaves open are marked READING):
  * f(P) = tr(A^T P B P^T) is the relaxed quadratic-assignment objective
    (Background, eq. (QAP)/(rQAP)); graph matching minimises -f (eq. (GM)),
    so GOAT maximises f over the Birkhoff polytope D.
  * grad f(P) = A P B^T + A^T P B (Alg. 3 step 1; Alg. 1 step 1).
  * The direction is the maximiser of tr(Q^T grad f) over D computed by
    entropic OT (Alg. 2 "LOT"; Alg. 3 step 2). Maximisation is done by
    negating the cost (Methods, "Doubly Stochastic Optimal Transport"), i.e.
    the Gibbs kernel is exp(+G/eps).
  * READING (regularisation): eps = eps_rel * max|G| (the paper's lambda
    is 1/eps; it recommends lambda >= 100 without saying whether the cost is
    normalised). eps_rel defaults to 0.03.
  * READING (Sinkhorn stop): the L-infinity row-marginal error of the current
    plan, measured after a column update (so columns are exact), checked from
    the second iteration on; rows are updated first.
  * READING (step): the paper's alpha in P <- alpha P + (1-alpha) Q is
    1 - t with P <- P + t (Q - P); t maximises the exact quadratic
    f(P + t(Q-P)) over [0, 1] (Alg. 3 step 3, "as in" seeded FAQ).
  * READING (FW stop): at fw_max iterations or on an exact stall (t == 0);
    an optional ||dP||_F / sqrt(n) < fw_tol test is off by default.
  * READING (final projection): perm = argmax over permutations of
    <Pi, P_final> by default (proj="P"); proj="GRAD" uses <Pi, grad f(P_final)>
    as printed in Alg. 3's return line.
  * READING (FAQ, the comparison system): Alg. 1 with an argmax direction
    (the maximisation form of its argmin steps), GOAT's exact step and stop
    rules, the final assignment on P. Used only to compare against GOAT.
  * READING (soft matching): the Discussion names vertex nomination as
    future work; nominate() ranks, per row of P, the columns by score (ties
    by column).
  * READING (device assignment): the quantised scores the device solves
    exactly are defined in quantised_scores().
  * READING (warm starts, not in the paper): a Sinkhorn solve may start from
    column potentials g0 other than 0 (the previous FW iteration's g, or the
    warm-start network's prediction, mlp_oracle.warm_start); the fixed point,
    the stop rule and the cap are unchanged.
  * READING (seeds, unequal sizes): see the section of seeded_problem().
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------- objective

def relaxed_objective(A, B, P) -> float:
    """f(P) = tr(A^T P B P^T) (Background, eq. (QAP) over D = eq. (rQAP))."""
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64); P = np.asarray(P, np.float64)
    return float(np.sum(A * (P @ B @ P.T)))


def qap_value(A, B, perm) -> float:
    """tr(A^T Pi B Pi^T) for the permutation matrix Pi[i, perm[i]] = 1, i.e.
    sum_ij A_ij B_{perm i, perm j}. Graph matching minimises its negation
    (eq. (GM))."""
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64)
    perm = np.asarray(perm)
    return float(np.sum(A * B[np.ix_(perm, perm)]))


def edge_disagreements(A, B, perm) -> float:
    """||A - Pi B Pi^T||_F^2 (Graph Matching Problem, eq. (1))."""
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64)
    perm = np.asarray(perm)
    D = A - B[np.ix_(perm, perm)]
    return float(np.sum(D * D))


def perm_matrix(perm) -> np.ndarray:
    n = len(perm)
    Pi = np.zeros((n, n))
    Pi[np.arange(n), np.asarray(perm)] = 1.0
    return Pi


# ----------------------------------------------------------------- gradient

def gradient(A, B, P) -> np.ndarray:
    """grad f(P) = A P B^T + A^T P B (Alg. 3 step 1)."""
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64); P = np.asarray(P, np.float64)
    return A @ P @ B.T + A.T @ P @ B


# ----------------------------------------------------------------- Sinkhorn

def _lse_rows(X) -> np.ndarray:
    """log sum_j exp(X_ij), max-shifted."""
    m = np.max(X, axis=1)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    return m_safe + np.log(np.sum(np.exp(X - m_safe[:, None]), axis=1))


@dataclass
class SinkhornResult:
    f: np.ndarray
    g: np.ndarray
    Q: np.ndarray
    iters: int          # number of completed column updates
    err: float          # max_i |sum_j Q_ij - 1| of the returned Q
    converged: bool


def log_sinkhorn_max(G, eps: float, tol: float = 1e-6, max_iter: int = 1000,
                     g0=None) -> SinkhornResult:
    """Entropic maximiser of tr(Q^T G) over the Birkhoff polytope
    (Alg. 2 "LOT" with the cost negated; Sinkhorn distance, eq. (5)).

    The Sinkhorn-Knopp fixed point on K = exp(G/eps) is run in the log
    domain on dual potentials f (rows) and g (columns):
        f_i = -eps * log sum_j exp((G_ij + g_j)/eps)     (row scaling)
        g_j = -eps * log sum_i exp((G_ij + f_i)/eps)     (column scaling)
    and Q_ij = exp((G_ij + f_i + g_j)/eps), which lies in U(1, 1) = D.
    Stop rule: see the module READING; iters counts column updates.
    """
    G = np.asarray(G, np.float64)
    n, m = G.shape
    g = np.zeros(m) if g0 is None else np.asarray(g0, np.float64).copy()
    f = np.zeros(n)
    iters = 0
    converged = False
    for k in range(max_iter):
        s = _lse_rows((G + g[None, :]) / eps)
        if k >= 1:
            err = float(np.max(np.abs(np.exp(f / eps + s) - 1.0)))
            if err <= tol:
                converged = True
                break
        f = -eps * s
        g = -eps * _lse_rows(((G + f[:, None]) / eps).T)
        iters += 1
    Q = np.exp((G + f[:, None] + g[None, :]) / eps)
    err = float(np.max(np.abs(Q.sum(axis=1) - 1.0)))
    return SinkhornResult(f, g, Q, iters, err, converged)


def sinkhorn_knopp(K, tol: float = 1e-12, max_iter: int = 100000) -> np.ndarray:
    """Plain Sinkhorn-Knopp scaling of a positive matrix to a doubly
    stochastic one (used to draw the random start K in P0 = (J + K)/2,
    GOAT section, random initialisations)."""
    K = np.asarray(K, np.float64)
    n = K.shape[0]
    r = np.ones(n)
    c = np.ones(n)
    for _ in range(max_iter):
        r = 1.0 / (K @ c)
        c = 1.0 / (K.T @ r)
        X = r[:, None] * K * c[None, :]
        if np.max(np.abs(X.sum(axis=1) - 1.0)) <= tol:
            return X
    return r[:, None] * K * c[None, :]


def barycenter(n: int) -> np.ndarray:
    """J = 1 1^T / n (Alg. 1 and Alg. 3 initialisation)."""
    return np.full((n, n), 1.0 / n)


def random_init(U) -> np.ndarray:
    """P0 = (J + K)/2 with K the Sinkhorn-Knopp scaling of a positive random
    matrix U (GOAT section, random initialisations)."""
    U = np.asarray(U, np.float64)
    return 0.5 * (barycenter(U.shape[0]) + sinkhorn_knopp(U))


# -------------------------------------------------------------- line search

@dataclass
class LineSearch:
    fP: float
    fQ: float
    c: float
    a: float
    b: float
    t: float
    dist2: float        # ||Q - P||_F^2


def linesearch(P, Q, GP, GQ) -> LineSearch:
    """Exact step of Alg. 3 step 3 (READING: t = 1 - alpha).

    f is quadratic, so with D = Q - P:
        f(P + tD) = f(P) + t <D, grad f(P)> + t^2 f(D)
    and <P, grad f(P)> = 2 f(P), f(D) = f(P) + f(Q) - <Q, grad f(P)>. Hence
    with fP = <P,GP>/2, fQ = <Q,GQ>/2, c = <Q,GP>:
        b = c - 2 fP,   a = fP + fQ - c,   f(P + tD) = fP + b t + a t^2.
    t maximises b t + a t^2 over [0, 1]: the vertex -b/(2a) clipped to
    [0, 1] when a < 0, else the better endpoint (t = 1 iff a + b > 0)."""
    P = np.asarray(P, np.float64); Q = np.asarray(Q, np.float64)
    GP = np.asarray(GP, np.float64); GQ = np.asarray(GQ, np.float64)
    fP = 0.5 * float(np.sum(P * GP))
    fQ = 0.5 * float(np.sum(Q * GQ))
    c = float(np.sum(Q * GP))
    a = fP + fQ - c
    b = c - 2.0 * fP
    if a < 0.0:
        t = min(max(-b / (2.0 * a), 0.0), 1.0)
    else:
        t = 1.0 if a + b > 0.0 else 0.0
    D = Q - P
    return LineSearch(fP, fQ, c, a, b, t, float(np.sum(D * D)))


# ----------------------------------------------------- linear assignment

def hungarian_max(M) -> np.ndarray:
    """perm maximising sum_i M[i, perm[i]] (the linear assignment of Alg. 3's
    return line and Alg. 1 step 2, a Hungarian method).

    Textbook shortest-augmenting-path Hungarian algorithm with row/column
    dual potentials on the cost C = -M, adding one row at a time; FP64.
    Among columns of equal reduced distance the lowest index is taken.
    """
    C = -np.asarray(M, np.float64)
    n = C.shape[0]
    INF = math.inf
    u = np.zeros(n + 1)           # row potentials (1-based, 0 = virtual)
    v = np.zeros(n + 1)           # column potentials
    p = np.zeros(n + 1, dtype=np.int64)    # p[j] = row matched to column j
    way = np.zeros(n + 1, dtype=np.int64)
    for i in range(1, n + 1):
        p[0] = i
        j0 = 0
        minv = np.full(n + 1, INF)
        used = np.zeros(n + 1, dtype=bool)
        while True:
            used[j0] = True
            i0 = p[j0]
            # reduced costs of row i0 to every free (unused) column
            cur = C[i0 - 1, :] - u[i0] - v[1:]
            free = ~used[1:]
            upd = free & (cur < minv[1:])
            minv[1:][upd] = cur[upd]
            way[1:][upd] = j0
            cand = np.where(free, minv[1:], INF)
            j1 = int(np.argmin(cand)) + 1     # lowest index among equal minima
            delta = cand[j1 - 1]
            used_idx = np.nonzero(used)[0]
            u[p[used_idx]] += delta
            v[used_idx] -= delta
            minv[1:][free] -= delta
            j0 = j1
            if p[j0] == 0:
                break
        while True:
            j1 = way[j0]
            p[j0] = p[j1]
            j0 = j1
            if j0 == 0:
                break
    perm = np.empty(n, dtype=np.int64)
    for j in range(1, n + 1):
        perm[p[j] - 1] = j - 1
    return perm


# ---------------------------------------------------------------- GOAT loop

@dataclass
class GoatOptions:
    eps_rel: float = 0.03
    sk_tol: float = 1e-6
    sk_max: int = 1000
    fw_max: int = 30
    fw_tol: float = 0.0
    proj: str = "P"           # "P" or "GRAD"
    # Sinkhorn start (READING, warm starts): "cold" g0 = 0 every iteration;
    # "prev" the previous iteration's g; "net" the warm-start network every
    # iteration; "net_prev" the network on the first iteration, then "prev".
    warm: str = "cold"
    stop_on_stall: bool = True   # False: run fw_max iterations even after t == 0
    # final assignment: "hungarian" (hungarian_max below) or "scipy" (SciPy's
    # exact solver for the same maximisation, for sizes where the plain
    # Python loop would take hours)
    lap: str = "hungarian"


@dataclass
class GoatResult:
    perm: np.ndarray
    score: float               # tr(A^T Pi B Pi^T) of the returned perm
    P: np.ndarray
    fw_iters: int
    history: list = field(default_factory=list)
    start: int = 0             # goat_restarts: index of the kept start


def sinkhorn_start(opt: GoatOptions, it: int, G, eps: float, g_prev, net):
    """Column potentials g0 that start iteration `it`'s Sinkhorn solve
    (READING, warm starts; the paper always starts cold). Any start leads to
    the same fixed point; only the number of sweeps to reach it changes.
    `net(G, eps)` returns the warm-start network's g0 (see
    mlp_oracle.warm_start)."""
    if opt.warm == "cold":
        return None
    if opt.warm == "prev" or (opt.warm == "net_prev" and it > 1):
        return g_prev
    if opt.warm in ("net", "net_prev"):
        if net is None:
            raise ValueError("a network start needs the network")
        return net(G, eps)
    raise ValueError(f"unknown warm start {opt.warm!r}")


def assign_max(M, how: str = "hungarian") -> np.ndarray:
    """perm maximising sum_i M[i, perm[i]]: hungarian_max, or SciPy's exact
    solver of the same problem."""
    if how == "hungarian":
        return hungarian_max(M)
    if how == "scipy":
        from scipy.optimize import linear_sum_assignment
        rows, cols = linear_sum_assignment(np.asarray(M, np.float64), maximize=True)
        perm = np.empty(len(rows), dtype=np.int64)
        perm[rows] = cols
        return perm
    raise ValueError(f"unknown assignment {how!r}")


def goat(A, B, P0=None, opt: GoatOptions | None = None, record: bool = False,
         net=None, keep_rows=None, callback=None) -> GoatResult:
    """Alg. 3 (GOAT): Frank-Wolfe on the relaxed problem with the LAP
    direction of FAQ (Alg. 1) replaced by LOT (Alg. 2), then one Hungarian
    projection. The gradient is recomputed plainly each iteration.
    `net`: the warm-start network for opt.warm "net" / "net_prev";
    `keep_rows`: with record, the history also keeps these rows of Q;
    `callback(history, P)`: with record, called after every iteration (for
    long runs that report as they go)."""
    opt = opt or GoatOptions()
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64)
    n = A.shape[0]
    P = barycenter(n) if P0 is None else np.asarray(P0, np.float64).copy()
    hist = []
    it = 0
    g_prev = None
    for it in range(1, opt.fw_max + 1):
        G = gradient(A, B, P)                                   # step 1
        gmax = float(np.max(np.abs(G)))
        eps = opt.eps_rel * gmax
        if eps == 0.0:
            Q = barycenter(n); sk_it = 0; sk_err = 0.0
        else:
            g0 = sinkhorn_start(opt, it, G, eps, g_prev, net)
            sk = log_sinkhorn_max(G, eps, opt.sk_tol, opt.sk_max, g0=g0)   # step 2
            Q, sk_it, sk_err = sk.Q, sk.iters, sk.err
            g_prev = sk.g
        GQ = gradient(A, B, Q)
        ls = linesearch(P, Q, G, GQ)                            # step 3
        P = P + ls.t * (Q - P)                                  # step 4
        delta = ls.t * math.sqrt(ls.dist2) / math.sqrt(n)
        if record:
            hist.append(dict(it=it, eps=eps, sk_iters=sk_it, sk_err=sk_err,
                             t=ls.t, a=ls.a, b=ls.b, fP=ls.fP, fQ=ls.fQ, c=ls.c,
                             f_next=ls.fP + ls.b * ls.t + ls.a * ls.t ** 2))
            if keep_rows is not None:
                hist[-1]["Q_rows"] = Q[np.asarray(keep_rows)].copy()
            if callback is not None:
                callback(hist, P)
        if (ls.t == 0.0 and opt.stop_on_stall) or (opt.fw_tol > 0.0 and delta < opt.fw_tol):
            break
    M = P if opt.proj == "P" else gradient(A, B, P)
    perm = assign_max(M, opt.lap)
    return GoatResult(perm, qap_value(A, B, perm), P, it, hist)


def goat_restarts(A, B, inits, opt: GoatOptions | None = None) -> GoatResult:
    """Several starts P0 (GOAT section, random initialisations); the
    permutation with the largest tr(A^T Pi B Pi^T) is kept, ties to the
    earliest start."""
    best = None
    for k, P0 in enumerate(inits):
        r = goat(A, B, P0, opt)
        r.start = k
        if best is None or r.score > best.score:
            best = r
    return best


def match_ratio(perm, truth) -> float:
    """Fraction of nodes aligned as planted (Results section)."""
    return float(np.mean(np.asarray(perm) == np.asarray(truth)))


# ---------------------------------------------------------------- seeds, unequal sizes

# READING (seeded / unequal-size GOAT): the paper applies Fishkind et al.'s
# modification of FAQ without printing it. Restated here from that method:
# seeded vertices come first in both graphs (seed i of A is matched to seed
# i of B), the other vertices follow in increasing order, and the smaller
# graph is padded with isolated dummy vertices ("naive" padding) or, for 0/1
# graphs, both graphs are first recentred to 2X - J ("adopted" padding, so
# that an edge to a dummy vertex is neither rewarded nor penalised). With
# blocks X11 (seeds), X12, X21, X22 and a doubly stochastic P on the
# non-seed block, Pi = diag(I, P) gives
#     tr(A^T Pi B Pi^T) = tr(A11^T B11) + <C, P> + tr(A22^T P B22 P^T),
#     C = A21 B21^T + A12^T B12,
# so the gradient is C + A22 P B22^T + A22^T P B22 and the exact step gains
# the linear term's share below.

@dataclass
class SeededProblem:
    A: np.ndarray          # n x n, seeds first, padded
    B: np.ndarray
    m: int                 # number of seeds
    order_A: np.ndarray    # position -> original A vertex (-1: dummy)
    order_B: np.ndarray


def seeded_problem(A, B, seeds_A=(), seeds_B=(), pad: str = "naive") -> SeededProblem:
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64)
    seeds_A = [int(v) for v in seeds_A]; seeds_B = [int(v) for v in seeds_B]
    if len(seeds_A) != len(seeds_B) or len(set(seeds_A)) != len(seeds_A) or len(set(seeds_B)) != len(seeds_B):
        raise ValueError("seeds must be two equally long lists of distinct vertices")
    if pad == "adopted":
        A = 2.0 * A - 1.0
        B = 2.0 * B - 1.0
    elif pad != "naive":
        raise ValueError("pad must be 'naive' or 'adopted'")
    nA, nB = A.shape[0], B.shape[0]
    n = max(nA, nB)

    def order(nx, seeds):
        sset = set(seeds)
        rest = [v for v in range(nx) if v not in sset]
        return np.array(seeds + rest + [-1] * (n - nx), dtype=np.int64)

    oA, oB = order(nA, seeds_A), order(nB, seeds_B)

    def arrange(X, o):
        Y = np.zeros((n, n))
        real = np.nonzero(o >= 0)[0]
        Y[np.ix_(real, real)] = X[np.ix_(o[real], o[real])]
        return Y

    return SeededProblem(arrange(A, oA), arrange(B, oB), len(seeds_A), oA, oB)


def seeded_linear_term(sp: SeededProblem) -> np.ndarray:
    m = sp.m
    A, B = sp.A, sp.B
    return A[m:, :m] @ B[m:, :m].T + A[:m, m:].T @ B[:m, m:]


def seeded_gradient(sp: SeededProblem, P) -> np.ndarray:
    m = sp.m
    A22, B22 = sp.A[m:, m:], sp.B[m:, m:]
    return seeded_linear_term(sp) + A22 @ P @ B22.T + A22.T @ P @ B22


def seeded_objective(sp: SeededProblem, P) -> float:
    """<C, P> + tr(A22^T P B22 P^T) (the seeded objective without its
    constant tr(A11^T B11))."""
    m = sp.m
    return float(np.sum(seeded_linear_term(sp) * P)) + relaxed_objective(sp.A[m:, m:], sp.B[m:, m:], P)


def seeded_linesearch(P, Q, GP, GQ, C) -> LineSearch:
    """Exact step for f(X) = <C, X> + q(X), q quadratic with gradient
    grad q(X) = G_X - C. With D = Q - P:
        f(P + tD) = f(P) + t <D, G_P> + t^2 q(D),
        q(D) = q(Q) - <Q, grad q(P)> + q(P)
             = <Q,G_Q>/2 - <Q,G_P> + <P,G_P>/2 + <Q - P, C>/2.
    fP and fQ are f(P) and f(Q) themselves."""
    P = np.asarray(P, np.float64); Q = np.asarray(Q, np.float64)
    qp, qq = float(np.sum(Q * GP)), float(np.sum(P * GP))
    a = 0.5 * float(np.sum(Q * GQ)) - qp + 0.5 * qq + 0.5 * float(np.sum((Q - P) * C))
    b = qp - qq
    if a < 0.0:
        t = min(max(-b / (2.0 * a), 0.0), 1.0)
    else:
        t = 1.0 if a + b > 0.0 else 0.0
    fP = 0.5 * qq + 0.5 * float(np.sum(P * C))
    fQ = 0.5 * float(np.sum(Q * GQ)) + 0.5 * float(np.sum(Q * C))
    return LineSearch(fP, fQ, qp, a, b, t, float(np.sum((Q - P) ** 2)))


@dataclass
class SeededResult:
    perm: np.ndarray       # A vertex -> B vertex, -1 if matched to a dummy
    score: float           # tr(A'^T Pi B'^T Pi^T) on the arranged (padded) graphs
    P: np.ndarray          # final P on the non-seed block
    fw_iters: int
    history: list = field(default_factory=list)


def goat_seeded(A, B, seeds_A=(), seeds_B=(), P0=None, opt: GoatOptions | None = None,
                pad: str = "naive", record: bool = False) -> SeededResult:
    """GOAT on the non-seed block of the seeded (and padded) problem: the
    loop of Alg. 3 with the seeded gradient and step; the final assignment
    maps the non-seed block, seeds map to each other."""
    opt = opt or GoatOptions()
    sp = seeded_problem(A, B, seeds_A, seeds_B, pad)
    n, m = sp.A.shape[0], sp.m
    k = n - m
    C = seeded_linear_term(sp)
    if k == 0:
        P = np.zeros((0, 0))
    else:
        P = barycenter(k) if P0 is None else np.asarray(P0, np.float64).copy()
    hist = []
    it = 0
    if k > 0:
        for it in range(1, opt.fw_max + 1):
            G = seeded_gradient(sp, P)
            gmax = float(np.max(np.abs(G)))
            eps = opt.eps_rel * gmax
            if eps == 0.0:
                Q = barycenter(k); sk_it = 0; sk_err = 0.0
            else:
                sk = log_sinkhorn_max(G, eps, opt.sk_tol, opt.sk_max)
                Q, sk_it, sk_err = sk.Q, sk.iters, sk.err
            GQ = seeded_gradient(sp, Q)
            ls = seeded_linesearch(P, Q, G, GQ, C)
            P = P + ls.t * (Q - P)
            delta = ls.t * math.sqrt(ls.dist2) / math.sqrt(k)
            if record:
                hist.append(dict(it=it, eps=eps, sk_iters=sk_it, sk_err=sk_err, t=ls.t, a=ls.a, b=ls.b,
                                 fP=ls.fP, fQ=ls.fQ, c=ls.c))
            if ls.t == 0.0 or (opt.fw_tol > 0.0 and delta < opt.fw_tol):
                break
        M = P if opt.proj == "P" else seeded_gradient(sp, P)
        inner = hungarian_max(M)
    else:
        inner = np.zeros(0, dtype=np.int64)
    pos = np.concatenate([np.arange(m), m + inner]).astype(np.int64)
    nA = int(np.sum(sp.order_A >= 0))
    perm = np.full(nA, -1, dtype=np.int64)
    for i in range(n):
        a = sp.order_A[i]
        if a >= 0:
            perm[a] = sp.order_B[pos[i]]
    score = float(np.sum(sp.A * sp.B[np.ix_(pos, pos)]))
    return SeededResult(perm, score, P, it, hist)


# ---------------------------------------------------------------- FAQ, nomination

def faq(A, B, P0=None, opt: GoatOptions | None = None, record: bool = False) -> GoatResult:
    """Alg. 1 (FAQ), the comparison system: the Frank-Wolfe loop of Alg. 3
    with the direction taken by an exact linear assignment on the gradient
    (a permutation matrix maximising <Q, grad f(P)>; SciPy's solver is the
    library step), the same exact step, and the final assignment on P.
    Oracle only: the device library implements GOAT."""
    from scipy.optimize import linear_sum_assignment
    opt = opt or GoatOptions()
    A = np.asarray(A, np.float64); B = np.asarray(B, np.float64)
    n = A.shape[0]
    P = barycenter(n) if P0 is None else np.asarray(P0, np.float64).copy()
    hist = []
    it = 0
    for it in range(1, opt.fw_max + 1):
        G = gradient(A, B, P)
        rows, cols = linear_sum_assignment(G, maximize=True)
        Q = np.zeros((n, n))
        Q[rows, cols] = 1.0
        GQ = gradient(A, B, Q)
        ls = linesearch(P, Q, G, GQ)
        P = P + ls.t * (Q - P)
        if record:
            hist.append(dict(it=it, t=ls.t, fP=ls.fP, fQ=ls.fQ, c=ls.c, direction=cols.copy()))
        delta = ls.t * math.sqrt(ls.dist2) / math.sqrt(n)
        if ls.t == 0.0 or (opt.fw_tol > 0.0 and delta < opt.fw_tol):
            break
    rows, cols = linear_sum_assignment(P if opt.proj == "P" else gradient(A, B, P), maximize=True)
    perm = np.empty(n, dtype=np.int64)
    perm[rows] = cols
    return GoatResult(perm, qap_value(A, B, perm), P, it, hist)


def nominate(P, k: int) -> np.ndarray:
    """Soft matching (vertex nomination, Discussion): for each vertex i of A
    the k vertices of B with the largest P[i, j], best first; equal values
    in increasing column order."""
    P = np.asarray(P, np.float64)
    n = P.shape[1]
    k = min(k, n)
    out = np.empty((P.shape[0], k), dtype=np.int64)
    for i in range(P.shape[0]):
        order = sorted(range(n), key=lambda j: (-P[i, j], j))
        out[i] = order[:k]
    return out


# ----------------------------------------------------- quantised assignment

def lap_resolution_bits(n: int) -> int:
    """READING (device assignment): the integer scores of the final
    assignment carry R = min(40, 55 - ceil(log2(n + 1))) bits."""
    return min(40, 55 - int(math.ceil(math.log2(n + 1))))


def quantised_scores(M) -> tuple[np.ndarray, int]:
    """The integer scores the device assignment maximises: with
    2^(e-1) <= max|M| < 2^e and s = R - 1 - e, c = rint(M 2^s) - min rint(M 2^s)
    (round half to even). Returns (c as int64, s)."""
    M = np.asarray(M, np.float64)
    R = lap_resolution_bits(M.shape[0])
    mx = float(np.max(np.abs(M)))
    e = int(np.frexp(mx)[1]) if mx > 0 else 0
    s = R - 1 - e
    q = np.rint(np.ldexp(M, s)).astype(np.int64)
    return q - q.min(), s


def lap_quantised(M) -> tuple[np.ndarray, int]:
    """An optimal assignment of the quantised scores (Alg. 3 return line on
    c) and its value sum_i c[i, perm i] (exact, integer)."""
    from scipy.optimize import linear_sum_assignment
    c, _ = quantised_scores(M)
    rows, cols = linear_sum_assignment(c, maximize=True)
    perm = np.empty(c.shape[0], dtype=np.int64)
    perm[rows] = cols
    return perm, int(c[rows, cols].sum())
