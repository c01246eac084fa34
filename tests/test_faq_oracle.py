"""Pins of the oracle's FAQ mode (Alg. 1, the comparison system) and of the
soft-matching output (nominate). CPU only.

FAQ: every direction is an optimal assignment of the gradient (brute force
over all permutations at n = 6), the exact step never lowers the objective,
iterates stay doubly stochastic, isomorphic pairs are matched exactly, and
on correlated SBM pairs below rho = 1 GOAT matches at least as well (the
paper's comparison on the three-block SBM of its first simulation).
nominate: k = 1 is numpy's first arg-max; k = cols is numpy's lexsort order
(score descending, column ascending); a permutation matrix nominates its own
permutation first.
Quantised assignment scores (the device assignment's integer problem): exact
on dyadic inputs, brute-force optimum at n = 7, and within n 2^-s of the
float optimum.
"""
import itertools

import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I

SBM3 = [[0.2, 0.01, 0.01], [0.01, 0.1, 0.01], [0.01, 0.01, 0.2]]


def _weighted(seed, n=6, sym=False):
    rng = np.random.default_rng(seed)
    A = rng.random((n, n))
    B = rng.random((n, n))
    if sym:
        A = A + A.T
        B = B + B.T
    return A, B


@pytest.mark.parametrize("seed,sym", [(1, False), (2, True), (3, False)])
def test_faq_directions_are_optimal_assignments(seed, sym):
    A, B = _weighted(seed, sym=sym)
    n = A.shape[0]
    r = O.faq(A, B, opt=O.GoatOptions(fw_max=8), record=True)
    perms = [np.array(p) for p in itertools.permutations(range(n))]
    P = O.barycenter(n)
    assert r.history
    for h in r.history:
        G = O.gradient(A, B, P)
        best = max(G[np.arange(n), p].sum() for p in perms)
        got = G[np.arange(n), h["direction"]].sum()
        assert got == pytest.approx(best, rel=1e-12, abs=1e-12)
        Q = O.perm_matrix(h["direction"])
        P = P + h["t"] * (Q - P)
    assert np.allclose(P, r.P, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [4, 5])
def test_faq_monotone_and_doubly_stochastic(seed):
    A, B = _weighted(seed, n=40, sym=True)
    r = O.faq(A, B, opt=O.GoatOptions(fw_max=25), record=True)
    fs = [h["fP"] for h in r.history]
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(fs, fs[1:]))
    assert all(0.0 <= h["t"] <= 1.0 for h in r.history)
    assert np.allclose(r.P.sum(0), 1.0, atol=1e-12) and np.allclose(r.P.sum(1), 1.0, atol=1e-12)
    assert r.P.min() >= -1e-15
    # the reported score is the objective of the returned permutation
    assert r.score == pytest.approx(O.relaxed_objective(A, B, O.perm_matrix(r.perm)), rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_faq_matches_isomorphic_sbm_exactly(seed):
    g = I.rho_sbm_pair([50, 50, 50], SBM3, 1.0, 9000 + seed)
    r = O.faq(g.A, g.B)
    assert O.match_ratio(r.perm, g.truth) == 1.0


def test_goat_at_least_faq_on_correlated_sbm():
    # n = 150, three blocks of 50 (first simulation of the paper), rho = 0.8:
    # FAQ from the barycenter lands near chance, GOAT on the planted matching
    g = I.rho_sbm_pair([50, 50, 50], SBM3, 0.8, 9002)
    rf = O.faq(g.A, g.B)
    rg = O.goat(g.A, g.B)
    mf = O.match_ratio(rf.perm, g.truth)
    mg = O.match_ratio(rg.perm, g.truth)
    assert mg >= mf
    assert mg == 1.0 and mf < 0.1


def test_nominate_k1_is_first_argmax():
    rng = np.random.default_rng(11)
    P = np.round(rng.random((30, 17)) * 8) / 8          # many ties
    got = O.nominate(P, 1)[:, 0]
    assert np.array_equal(got, np.argmax(P, axis=1))


@pytest.mark.parametrize("rows,cols", [(5, 9), (12, 12), (3, 40)])
def test_nominate_full_order_is_lexsort(rows, cols):
    rng = np.random.default_rng(rows * 100 + cols)
    P = np.round(rng.random((rows, cols)) * 5) / 5
    got = O.nominate(P, cols)
    for i in range(rows):
        want = np.lexsort((np.arange(cols), -P[i]))
        assert np.array_equal(got[i], want)
    # a prefix of the full order
    assert np.array_equal(O.nominate(P, 3), got[:, :3])


def test_nominate_permutation_matrix_first():
    perm = np.random.default_rng(3).permutation(25)
    P = O.perm_matrix(perm)
    top = O.nominate(P, 2)
    assert np.array_equal(top[:, 0], perm)
    # the runner-up is the smallest other column (all zeros tie)
    assert np.array_equal(top[:, 1], np.where(perm == 0, 1, 0))


# ------------------------------------------------- quantised assignment scores

def test_quantised_scores_exact_on_dyadic_input():
    # scores that are multiples of 2^-s are mapped by the affine map exactly
    rng = np.random.default_rng(21)
    n = 40
    M = rng.integers(-1000, 1000, size=(n, n)).astype(np.float64) / 1024.0
    c, s = O.quantised_scores(M)
    R = O.lap_resolution_bits(n)
    assert R == min(40, 55 - 6)
    mx = np.abs(M).max()
    assert 2.0 ** (R - 2) <= mx * 2.0 ** s < 2.0 ** (R - 1)
    assert np.array_equal(c, (M * 2.0 ** s - M.min() * 2.0 ** s).astype(np.int64))
    assert c.min() == 0 and c.max() <= 2 ** R


def test_lap_quantised_optimum_by_brute_force():
    rng = np.random.default_rng(22)
    M = rng.random((7, 7))
    perm, val = O.lap_quantised(M)
    c, _ = O.quantised_scores(M)
    best = max(int(c[np.arange(7), list(p)].sum()) for p in itertools.permutations(range(7)))
    assert val == best == int(c[np.arange(7), perm].sum())


def test_quantised_assignment_near_float_optimum():
    # on M itself the quantised optimum loses at most n 2^-s
    rng = np.random.default_rng(23)
    n = 60
    M = rng.random((n, n)) ** 6
    perm, _ = O.lap_quantised(M)
    _, s = O.quantised_scores(M)
    fperm = O.hungarian_max(M)
    best = M[np.arange(n), fperm].sum()
    assert M[np.arange(n), perm].sum() >= best - n * 2.0 ** -s
