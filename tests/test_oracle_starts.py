"""Pins of the oracle's starting points: the random start P0 = (J + K)/2
(GOAT section, random initialisations), the choice among restarts, and the
Sinkhorn warm starts (the previous iteration's potentials, the warm-start
network). CPU only; each pin is a fact fixed by the mathematics, not a
re-run of the same code."""
import itertools

import numpy as np
import pytest

from oracle import goat_oracle as O
from oracle import mlp_oracle as M
from paper_2111_05366_amd import inputs as I


# ------------------------------------------------------------ random start

@pytest.mark.parametrize("n", [3, 7, 40])
def test_random_init_is_half_barycenter_plus_scaled_U(n):
    """2 (P0 - J/2) = K must be doubly stochastic and a diagonal scaling of
    U, i.e. keep every cross-ratio U_ij U_kl / (U_il U_kj). Returning K alone,
    J alone or an unscaled mix fails one of the two."""
    U = I.uniform_matrix(n, 70 + n).astype(np.float64) + 0.05
    P0 = O.random_init(U)
    K = 2.0 * (P0 - 0.5 * O.barycenter(n))
    assert np.allclose(K.sum(axis=0), 1.0, atol=1e-11)
    assert np.allclose(K.sum(axis=1), 1.0, atol=1e-11)
    assert np.all(K > 0)
    rng = np.random.default_rng(n)
    for _ in range(20):
        i, k = rng.choice(n, 2, replace=False)
        j, l = rng.choice(n, 2, replace=False)
        want = U[i, j] * U[k, l] / (U[i, l] * U[k, j])
        got = K[i, j] * K[k, l] / (K[i, l] * K[k, j])
        assert got == pytest.approx(want, rel=1e-9)


def test_random_init_two_by_two_closed_form():
    """For 2 x 2 a doubly stochastic K is [[x, 1-x], [1-x, x]], and the
    cross-ratio fixes x: (x / (1-x))^2 = U00 U11 / (U01 U10)."""
    U = np.array([[0.3, 0.9], [0.5, 0.2]])
    r = np.sqrt(U[0, 0] * U[1, 1] / (U[0, 1] * U[1, 0]))
    x = r / (1.0 + r)
    want = 0.5 * (np.full((2, 2), 0.5) + np.array([[x, 1 - x], [1 - x, x]]))
    assert np.allclose(O.random_init(U), want, atol=1e-12)


# ---------------------------------------------------------------- restarts

def _brute_force_qap(A, B):
    n = A.shape[0]
    return max(O.qap_value(A, B, p) for p in itertools.permutations(range(n)))


def test_restarts_keep_best_score_with_earliest_tie():
    """goat_restarts returns the start with the largest tr(A^T Pi B Pi^T),
    the first such start on a tie. A cycle graph matched with itself has
    every rotation and reflection as an optimum, so different starts end on
    different permutations of equal score."""
    n = 6
    A = np.zeros((n, n))
    for i in range(n):
        A[i, (i + 1) % n] = A[(i + 1) % n, i] = 1.0
    opt = O.GoatOptions(sk_max=300, fw_max=30)
    inits = [O.random_init(I.uniform_matrix(n, 500 + r).astype(np.float64)) for r in range(6)]
    runs = [O.goat(A, A, P0=P0, opt=opt) for P0 in inits]
    best = O.goat_restarts(A, A, inits, opt)
    scores = [r.score for r in runs]
    k = int(np.argmax(scores))                       # numpy's argmax: first maximum
    assert best.start == k
    assert best.score == max(scores)
    assert list(best.perm) == list(runs[k].perm)
    # the optimum of the cycle is 2n (every edge kept), reached by brute force
    assert _brute_force_qap(A, A) == 2 * n
    # a tie: the same starts in reverse order keep the first of the reversed list
    tied = [i for i, s in enumerate(scores) if s == max(scores)]
    rev = O.goat_restarts(A, A, inits[::-1], opt)
    assert rev.start == len(inits) - 1 - tied[-1]


def test_restarts_reach_brute_force_optimum_on_isomorphic_pairs():
    for seed in range(3):
        g = I.rho_er_pair(7, 0.4, 1.0, 4000 + seed)
        inits = [O.random_init(I.uniform_matrix(7, 600 + 10 * seed + r).astype(np.float64)) for r in range(8)]
        best = O.goat_restarts(g.A, g.B, inits, O.GoatOptions(sk_max=300))
        assert best.score == _brute_force_qap(g.A.astype(float), g.B.astype(float))


# ------------------------------------------------------------- warm starts

def _problem(n, seed):
    g = I.rho_er_pair(n, 0.2, 0.9, seed)
    P = O.random_init(I.uniform_matrix(n, seed + 1).astype(np.float64))
    return g, O.gradient(g.A.astype(float), g.B.astype(float), P)


def test_converged_warm_start_reaches_cold_fixed_point():
    """Sinkhorn's fixed point does not depend on the start (the scaling of a
    positive matrix to a doubly stochastic one is unique): any g0 solved to
    a tight tolerance gives the cold start's Q."""
    g, G = _problem(40, 31)
    eps = 0.05 * float(np.max(np.abs(G)))
    cold = O.log_sinkhorn_max(G, eps, tol=1e-13, max_iter=20000)
    rng = np.random.default_rng(2)
    warm = O.log_sinkhorn_max(G, eps, tol=1e-13, max_iter=20000, g0=rng.normal(size=40) * eps * 3)
    assert cold.converged and warm.converged
    assert np.max(np.abs(cold.Q - warm.Q)) <= 1e-10


def _lse_network():
    """Weights of a 4-128-128-1 ReLU network that outputs minus its fourth
    input: y = relu(-x4) - relu(x4)."""
    p = {k: np.zeros(s) for k, s in
         dict(W1=(M.H, M.NFEAT), b1=(M.H,), W2=(M.H, M.H), b2=(M.H,), W3=(1, M.H), b3=(1,)).items()}
    p["W1"][0, 3] = 1.0
    p["W1"][1, 3] = -1.0
    p["W2"][0, 0] = 1.0
    p["W2"][1, 1] = 1.0
    p["W3"][0, 0] = -1.0
    p["W3"][0, 1] = 1.0
    flat = np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])
    return flat


def test_network_start_equals_column_update_from_zero_rows():
    """A network that returns minus the centred log-mean-exp feature starts
    Sinkhorn at g0_j = -eps LSE_i(G_ij / eps) + const, the column update from
    f = 0. The constant is a gauge shift (f + c, g - c leaves Q unchanged),
    so after k sweeps the plan equals that of a solve started from the
    column update computed directly."""
    g, G = _problem(30, 41)
    eps = 0.03 * float(np.max(np.abs(G)))
    net = M.network(_lse_network())
    g0 = net(G, eps)
    X = G / eps
    mx = X.max(axis=0)
    direct = -eps * (mx + np.log(np.exp(X - mx).sum(axis=0)))
    assert np.ptp(g0 - direct) <= 1e-9 * eps            # equal up to one constant
    for k in (1, 5, 40):
        a = O.log_sinkhorn_max(G, eps, tol=0.0, max_iter=k, g0=g0)
        b = O.log_sinkhorn_max(G, eps, tol=0.0, max_iter=k, g0=direct)
        assert np.max(np.abs(a.Q - b.Q)) <= 1e-12


def test_unpack_layout():
    flat = np.arange(M.H * M.NFEAT + M.H + M.H * M.H + M.H + M.H + 1, dtype=np.float32)
    p = M.unpack(flat)
    assert p["W1"][2, 3] == 2 * 4 + 3
    assert p["b1"][0] == M.H * M.NFEAT
    assert p["W2"][1, 0] == M.H * M.NFEAT + M.H + M.H
    assert p["b3"][0] == flat[-1]
    with pytest.raises(ValueError):
        M.unpack(flat[:-1])


def test_goat_warm_modes_pass_the_right_start():
    """warm="prev" starts iteration k + 1 from iteration k's g; "net_prev"
    starts iteration 1 from the network and later ones like "prev"; with
    converged solves every mode follows the cold trajectory."""
    g = I.rho_er_pair(24, 0.3, 0.9, 51)
    calls = []

    def net(G, eps):
        calls.append(eps)
        return np.zeros(G.shape[1])

    tight = dict(sk_tol=1e-12, sk_max=20000, fw_max=4, stop_on_stall=False)
    cold = O.goat(g.A, g.B, opt=O.GoatOptions(**tight), record=True)
    for warm in ("prev", "net", "net_prev"):
        calls.clear()
        r = O.goat(g.A, g.B, opt=O.GoatOptions(warm=warm, **tight), record=True, net=net)
        assert len(calls) == {"prev": 0, "net": 4, "net_prev": 1}[warm]
        for h, c in zip(r.history, cold.history):
            assert h["fP"] == pytest.approx(c["fP"], rel=1e-9)
            assert h["t"] == pytest.approx(c["t"], abs=1e-7)
    # with a loose cap the previous potentials change the capped solve
    loose = dict(sk_tol=1e-12, sk_max=3, fw_max=3, stop_on_stall=False)
    a = O.goat(g.A, g.B, opt=O.GoatOptions(**loose), record=True)
    b = O.goat(g.A, g.B, opt=O.GoatOptions(warm="prev", **loose), record=True)
    assert a.history[0]["fQ"] == b.history[0]["fQ"]      # the first solve starts cold in both
    assert a.history[1]["fQ"] != b.history[1]["fQ"]
