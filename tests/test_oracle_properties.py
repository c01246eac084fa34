"""Property-based pins of the oracle (random small inputs drawn by
hypothesis). Each property follows from the definitions, not from the
oracle's own code: the gradient of the quadratic objective is linear in P
and f(P) = <P, grad f(P)> / 2 (Background, eq. (rQAP); Alg. 3 step 1); the
exact step maximises f along the segment (Alg. 3 step 3); a converged
Sinkhorn plan has unit marginals and the cross-ratios of the Gibbs kernel
(Alg. 2); the quantised scores of the device assignment are a monotone map
into [0, 2^R]; nominations are ordered and free of duplicates. CPU only."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import goat_oracle as O

SET = settings(max_examples=25, deadline=None)


def _mats(seed, n, sym):
    rng = np.random.default_rng(seed)
    A = rng.random((n, n))
    B = rng.random((n, n))
    if sym:
        A, B = A + A.T, B + B.T
    return A, B


def _ds(seed, n):
    return O.sinkhorn_knopp(np.random.default_rng(seed).random((n, n)) + 0.05)


@SET
@given(seed=st.integers(0, 10_000), n=st.integers(2, 12), sym=st.booleans(),
       a=st.floats(-2, 2), b=st.floats(-2, 2))
def test_gradient_linear_and_objective_identity(seed, n, sym, a, b):
    A, B = _mats(seed, n, sym)
    P, Q = _ds(seed + 1, n), _ds(seed + 2, n)
    lhs = O.gradient(A, B, a * P + b * Q)
    rhs = a * O.gradient(A, B, P) + b * O.gradient(A, B, Q)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-10)
    assert O.relaxed_objective(A, B, P) == pytest.approx(0.5 * np.sum(P * O.gradient(A, B, P)), rel=1e-12)


@SET
@given(seed=st.integers(0, 10_000), n=st.integers(2, 10), sym=st.booleans())
def test_exact_step_beats_every_grid_point(seed, n, sym):
    A, B = _mats(seed, n, sym)
    P, Q = _ds(seed + 3, n), _ds(seed + 4, n)
    ls = O.linesearch(P, Q, O.gradient(A, B, P), O.gradient(A, B, Q))
    assert 0.0 <= ls.t <= 1.0
    f_t = O.relaxed_objective(A, B, P + ls.t * (Q - P))
    for s in np.linspace(0.0, 1.0, 41):
        assert f_t >= O.relaxed_objective(A, B, P + s * (Q - P)) - 1e-9 * max(1.0, abs(f_t))


@SET
@given(seed=st.integers(0, 10_000), n=st.integers(2, 9), eps=st.floats(0.2, 2.0))
def test_sinkhorn_marginals_and_cross_ratio(seed, n, eps):
    G = np.random.default_rng(seed).standard_normal((n, n))
    r = O.log_sinkhorn_max(G, eps, tol=1e-10, max_iter=20000)
    Q = r.Q
    assert np.allclose(Q.sum(1), 1.0, atol=1e-8) and np.allclose(Q.sum(0), 1.0, atol=1e-8)
    i, j, k, l = 0, 1, n - 1, 0
    if n >= 2 and i != k and j != l:
        lhs = np.log(Q[i, j]) + np.log(Q[k, l]) - np.log(Q[i, l]) - np.log(Q[k, j])
        assert lhs == pytest.approx((G[i, j] + G[k, l] - G[i, l] - G[k, j]) / eps, abs=1e-8)


@SET
@given(seed=st.integers(0, 10_000), n=st.integers(2, 40), scale=st.floats(1e-6, 1e6), shift=st.floats(-1, 1))
def test_quantised_scores_monotone_in_range(seed, n, scale, shift):
    M = ((np.random.default_rng(seed).random((n, n)) + shift) * scale).astype(np.float32).astype(np.float64)
    c, _ = O.quantised_scores(M)
    R = O.lap_resolution_bits(n)
    assert c.min() == 0 and c.max() <= 2 ** R
    order = np.argsort(M, axis=None, kind="stable")
    assert np.all(np.diff(c.ravel()[order]) >= 0)


@SET
@given(seed=st.integers(0, 10_000), rows=st.integers(1, 12), cols=st.integers(1, 30), k=st.integers(1, 30))
def test_nominations_ordered_and_distinct(seed, rows, cols, k):
    P = np.round(np.random.default_rng(seed).random((rows, cols)) * 6) / 6
    nom = O.nominate(P, k)
    kk = min(k, cols)
    assert nom.shape == (rows, kk)
    for i in range(rows):
        assert len(set(nom[i].tolist())) == kk
        vals = P[i, nom[i]]
        assert np.all(np.diff(vals) <= 0)
        # nothing outside the nominations beats the last one
        rest = np.setdiff1d(np.arange(cols), nom[i])
        if rest.size:
            assert P[i, rest].max() <= vals[-1]
