"""Pins of the seeded / unequal-size oracle (goat_seeded): the seeded
gradient is a block of the unseeded gradient, the exact step matches the
full objective along the segment, no seeds reduce to plain GOAT, and planted
matchings are recovered. CPU only."""
import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I


def _random_problem(seed, n=23, m=5, weighted=True):
    rng = np.random.default_rng(seed)
    A = rng.random((n, n)) if weighted else (rng.random((n, n)) < 0.3).astype(float)
    B = rng.random((n, n)) if weighted else (rng.random((n, n)) < 0.3).astype(float)
    seedsA = list(rng.choice(n, size=m, replace=False))
    seedsB = list(rng.choice(n, size=m, replace=False))
    return A, B, seedsA, seedsB


def _ds(k, seed):
    return O.sinkhorn_knopp(np.random.default_rng(seed).random((k, k)) + 0.05)


@pytest.mark.parametrize("m", [0, 1, 5, 12])
def test_seeded_gradient_is_block_of_full_gradient(m):
    A, B, sA, sB = _random_problem(100 + m, m=m)
    sp = O.seeded_problem(A, B, sA, sB)
    k = sp.A.shape[0] - m
    P = _ds(k, 7)
    Pi = np.eye(sp.A.shape[0])
    Pi[m:, m:] = P
    full = O.gradient(sp.A, sp.B, Pi)
    assert np.allclose(O.seeded_gradient(sp, P), full[m:, m:], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [0, 3, 9])
def test_seeded_step_matches_full_objective(m):
    A, B, sA, sB = _random_problem(200 + m, m=m)
    sp = O.seeded_problem(A, B, sA, sB)
    n = sp.A.shape[0]
    k = n - m
    P, Q = _ds(k, 8), _ds(k, 9)
    C = O.seeded_linear_term(sp)
    ls = O.seeded_linesearch(P, Q, O.seeded_gradient(sp, P), O.seeded_gradient(sp, Q), C)
    const = float(np.sum(sp.A[:m, :m] * sp.B[:m, :m]))
    for t in (0.0, 0.3, 0.7, 1.0):
        Pi = np.eye(n)
        Pi[m:, m:] = P + t * (Q - P)
        full = O.relaxed_objective(sp.A, sp.B, Pi) - const
        assert full == pytest.approx(ls.fP + ls.b * t + ls.a * t * t, rel=1e-12, abs=1e-9)
    assert ls.fP == pytest.approx(O.seeded_objective(sp, P), rel=1e-12)
    assert ls.fQ == pytest.approx(O.seeded_objective(sp, Q), rel=1e-12)


def test_no_seeds_is_plain_goat():
    g = I.rho_er_pair(40, 0.15, 0.8, 21)
    opt = O.GoatOptions(sk_max=500, fw_max=5)
    rs = O.goat_seeded(g.A, g.B, opt=opt, record=True)
    rg = O.goat(g.A, g.B, opt=opt, record=True)
    assert len(rs.history) == len(rg.history)
    for a, b in zip(rs.history, rg.history):
        assert a["fP"] == pytest.approx(b["fP"], rel=1e-12)
        assert a["t"] == pytest.approx(b["t"], abs=1e-12)
    assert list(rs.perm) == list(rg.perm)


def test_seeds_recover_isomorphic_pair():
    g = I.rho_er_pair(60, 0.15, 1.0, 5)
    sA = [0, 7, 13, 22, 40]
    sB = [int(g.truth[v]) for v in sA]
    r = O.goat_seeded(g.A, g.B, sA, sB, opt=O.GoatOptions(sk_max=500))
    assert list(r.perm) == list(g.truth)
    assert r.score == pytest.approx(O.qap_value(g.A, g.B, r.perm))


def test_all_seeds_is_the_seed_map():
    g = I.rho_er_pair(12, 0.3, 0.5, 6)
    sA = list(range(12))
    sB = list(np.random.default_rng(1).permutation(12))
    r = O.goat_seeded(g.A, g.B, sA, sB)
    assert r.fw_iters == 0
    assert list(r.perm) == [int(v) for v in sB]


@pytest.mark.parametrize("pad,m", [("adopted", 0), ("naive", 4), ("adopted", 8)])
def test_unequal_sizes_recover_induced_subgraph(pad, m):
    """A is the subgraph of B induced on 45 of its 60 vertices."""
    g = I.rho_er_pair(60, 0.2, 1.0, 11)
    sub = np.random.default_rng(3).choice(60, size=45, replace=False)
    A = g.B[np.ix_(sub, sub)]
    sA = list(range(m))
    sB = [int(sub[i]) for i in sA]
    r = O.goat_seeded(A, g.B, sA, sB, opt=O.GoatOptions(sk_max=500), pad=pad)
    assert list(r.perm) == [int(v) for v in sub]


def test_unequal_sizes_larger_first_graph_leaves_dummies_unmatched():
    g = I.rho_er_pair(30, 0.2, 1.0, 12)
    sub = np.arange(24)
    B = g.A[np.ix_(sub, sub)]
    r = O.goat_seeded(g.A, B, pad="adopted", opt=O.GoatOptions(sk_max=500))
    real = r.perm[r.perm >= 0]
    assert len(real) == 24 and len(set(real.tolist())) == 24
    assert np.sum(r.perm < 0) == 6
