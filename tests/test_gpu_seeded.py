"""Seeded and unequal-size GOAT on the device (goat_solve_seeded) against
the FP64 seeded oracle (goat_seeded) and planted matchings."""
import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "fp8"])
def test_seeded_matches_oracle(G, prec):
    g = I.rho_er_pair(80, 0.12, 0.8, 31)
    sA = [3, 17, 29, 44, 60, 71]
    sB = [int(g.truth[v]) for v in sA]
    r = G.solve_seeded(dev(g.A), dev(g.B), sA, sB, prec=prec, sk_max=500)
    ref = O.goat_seeded(g.A, g.B, sA, sB, opt=O.GoatOptions(sk_max=500), record=True)
    print(f"seeded {prec}: fw {len(r.history)} vs {ref.fw_iters}, match {np.mean(r.perm == g.truth):.4f} "
          f"vs {np.mean(ref.perm == g.truth):.4f}")
    for f in range(min(3, len(r.history), len(ref.history))):
        assert r.history[f]["fP"] == pytest.approx(ref.history[f]["fP"], rel=1e-5)
        assert r.history[f]["c"] == pytest.approx(ref.history[f]["c"], rel=1e-5)
        assert r.history[f]["t"] == pytest.approx(ref.history[f]["t"], abs=1e-4)
    assert abs(np.mean(r.perm == g.truth) - np.mean(ref.perm == g.truth)) <= 0.0125   # one vertex of 80
    for i, v in enumerate(sA):
        assert r.perm[v] == sB[i]


def test_no_seeds_equals_plain_solver(G):
    g = I.rho_er_pair(70, 0.12, 0.8, 32)
    A, B = dev(g.A), dev(g.B)
    r = G.solve_seeded(A, B, sk_max=400, fw_max=6, stop_on_stall=0)
    p = G.solve(A, B, sk_max=400, fw_max=6, stop_on_stall=0)
    assert r.history == p.history
    assert list(r.perm) == list(p.perm)


def test_seeds_recover_isomorphic_pair(G):
    g = I.rho_er_pair(100, 0.1, 1.0, 33)
    sA = [1, 20, 55, 70, 99]
    sB = [int(g.truth[v]) for v in sA]
    r = G.solve_seeded(dev(g.A), dev(g.B), sA, sB, sk_max=500)
    assert list(r.perm) == list(g.truth)
    assert r.stats.score == pytest.approx(O.qap_value(g.A, g.B, r.perm))


@pytest.mark.parametrize("pad,m", [("adopted", 0), ("naive", 4), ("adopted", 8)])
def test_unequal_sizes_recover_induced_subgraph(G, pad, m):
    g = I.rho_er_pair(60, 0.2, 1.0, 11)
    sub = np.random.default_rng(3).choice(60, size=45, replace=False)
    A = g.B[np.ix_(sub, sub)]
    sA = list(range(m))
    sB = [int(sub[i]) for i in sA]
    r = G.solve_seeded(dev(A), dev(g.B), sA, sB, pad=pad, sk_max=500)
    ref = O.goat_seeded(A, g.B, sA, sB, opt=O.GoatOptions(sk_max=500), pad=pad)
    assert list(r.perm) == [int(v) for v in sub] == list(ref.perm)


def test_larger_first_graph_leaves_dummies_unmatched(G):
    g = I.rho_er_pair(30, 0.2, 1.0, 12)
    B = g.A[:24, :24]
    r = G.solve_seeded(dev(g.A), dev(B), pad="adopted", sk_max=500)
    real = r.perm[r.perm >= 0]
    assert len(real) == 24 and len(set(real.tolist())) == 24
    assert int(np.sum(r.perm < 0)) == 6


def test_all_seeds_is_the_seed_map(G):
    g = I.rho_er_pair(12, 0.3, 0.5, 6)
    sB = np.random.default_rng(1).permutation(12)
    r = G.solve_seeded(dev(g.A), dev(g.B), list(range(12)), list(sB))
    assert list(r.perm) == [int(v) for v in sB]


def test_bad_seeds_rejected(G):
    g = I.rho_er_pair(20, 0.3, 0.5, 7)
    with pytest.raises(G.GoatError):
        G.solve_seeded(dev(g.A), dev(g.B), [1, 1], [2, 3])
    with pytest.raises(G.GoatError):
        G.solve_seeded(dev(g.A), dev(g.B), [1, 25], [2, 3])


def test_seeded_sbm_experiment_shape(G):
    """A small version of the paper's seeded experiment: rho-SBM with three
    equal blocks, n = 300, block probabilities [[.7,.3,.4],[.3,.7,.3],
    [.4,.3,.7]], rho = 0.6: more seeds do not lower the match ratio, and
    30 seeds recover most of the planted matching."""
    bp = [[0.7, 0.3, 0.4], [0.3, 0.7, 0.3], [0.4, 0.3, 0.7]]
    g = I.rho_sbm_pair([100, 100, 100], bp, 0.6, 41)
    A, B = dev(g.A), dev(g.B)
    rng = np.random.default_rng(2)
    order = rng.permutation(300)
    ratios = []
    for m in (0, 10, 30):
        sA = list(order[:m])
        sB = [int(g.truth[v]) for v in sA]
        r = G.solve_seeded(A, B, sA, sB, sk_max=1000)
        free = np.setdiff1d(np.arange(300), sA)
        ratios.append(float(np.mean(r.perm[free] == g.truth[free])))
    print(f"seeded SBM rho=0.6: match ratio on non-seeds for m = 0, 10, 30: {ratios}")
    assert ratios[2] >= ratios[0]
    assert ratios[2] >= 0.8
