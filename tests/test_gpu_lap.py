"""The final assignment on the device (goat_lap_device) against the oracle's
assignment of the same quantised scores: the returned map is a permutation
and its integer score equals the oracle's optimum exactly (several optimal
permutations may exist, so the value is compared, not the map); the shift s
is the oracle's. Cases: uniform, heavily tied, negative, near-permutation
and doubly stochastic scores, aligned and unaligned leading dimensions,
n = 2 .. 4000, the all-equal and one-vertex cases, goat_solve with the
device assignment, a planted permutation at n = 10,000, and the round cap.
"""
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


def _scores(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        M = rng.random((n, n))
    elif kind == "ties":
        M = np.floor(rng.random((n, n)) * 4) / 4
    elif kind == "negative":
        M = -rng.uniform(100, 150, (n, n))
    elif kind == "normal":
        M = rng.standard_normal((n, n))
    elif kind == "nearperm":
        M = rng.random((n, n)) * 1e-3 / n
        M[np.arange(n), rng.permutation(n)] += 0.9
    elif kind == "flat":
        # nearly uniform, like a solver iterate far from a permutation
        M = (1.0 + 0.05 * rng.standard_normal((n, n))) / n
    elif kind == "ds":
        X = rng.random((n, n)) ** 8
        M = O.sinkhorn_knopp(X + 1e-12, tol=1e-10)
    return M.astype(np.float32)


def _device(M, ld=None):
    n = M.shape[0]
    ld = n if ld is None else ld
    buf = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.as_tensor(M, device="cuda")
    return buf[:, :n]


def _check(G, M, ld=None, precompute=True):
    n = M.shape[0]
    perm, st = G.lap_device(_device(M, ld), precompute=precompute)
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    c, s = O.quantised_scores(M.astype(np.float64))
    _, best = O.lap_quantised(M.astype(np.float64))
    assert int(c[np.arange(n), perm].sum()) == best
    if n > 1 and c.max() > 0:
        assert st.shift == s and st.resolution_bits == O.lap_resolution_bits(n)
    return perm, st


@pytest.mark.parametrize("kind,n,ld", [
    ("uniform", 2, None), ("uniform", 3, None), ("ties", 64, None), ("normal", 257, None),
    ("uniform", 1000, None), ("negative", 1000, 1003), ("ties", 777, 780), ("ds", 1500, None),
    ("nearperm", 2001, 2005), ("uniform", 4000, None),
])
def test_lap_device_parity(G, kind, n, ld):
    print(f"lap_device {kind} n={n} ld={ld}", flush=True)
    M = _scores(kind, n, 31 * n + len(kind))
    perm, st = _check(G, M, ld)
    print(f"  rounds {st.rounds}, tail bids {st.tail_bids}, phases {st.phases}", flush=True)
    # the minimum workspace converts the scores in every scan: same bids,
    # same permutation
    perm_min, st_min = _check(G, M, ld, precompute=False)
    assert np.array_equal(perm, perm_min)
    assert (st.rounds, st.tail_bids, st.phases) == (st_min.rounds, st_min.tail_bids, st_min.phases)


_LISTS_OFF = """
import sys, json
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2111_05366_amd import goat
M = torch.as_tensor(np.load(sys.argv[2]), device="cuda")
perm, st = goat.lap_device(M)
np.save(sys.argv[3], perm.cpu().numpy())
print(json.dumps([st.rounds, st.tail_bids, st.phases, st.list_bids, st.skipped_phases]))
"""


@pytest.mark.parametrize("kind,n,switch", [("ds", 1500, "GOAT_LAP_LISTS=0"), ("flat", 2000, "GOAT_LAP_LISTS=0"),
                                           ("flat", 2000, "GOAT_LAP_SEQ_GLOBAL=1"),
                                           ("nearperm", 2001, "GOAT_LAP_SKIP_IDLE=0"),
                                           ("ds", 1500, "GOAT_LAP_SKIP_IDLE=0")])
def test_lap_device_variants_change_nothing(G, kind, n, switch, tmp_path):
    # a bid decided by the row's candidate list is the bid a full scan
    # gives; the sequential kernel's state in global memory (the path taken
    # above about 10,000 vertices) gives the bids of the LDS state; a phase
    # passed over because its filter would keep every pair changes nothing:
    # with the switch set (in a fresh process, switches are read once)
    # every count and the permutation are the same
    import json
    import os
    import subprocess
    import sys
    M = _scores(kind, n, 5 * n + 1)
    perm, st = _check(G, M)
    print(f"{kind} n={n}: tail bids {st.tail_bids}, decided by lists {st.list_bids}", flush=True)
    if switch == "GOAT_LAP_LISTS=0":
        assert st.list_bids > 0
    np.save(tmp_path / "M.npy", M)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    key, val = switch.split("=")
    env = dict(os.environ, **{key: val})
    out = subprocess.run([sys.executable, "-c", _LISTS_OFF, root, str(tmp_path / "M.npy"), str(tmp_path / "p.npy")],
                         env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rounds, tail, phases, listed, skipped = json.loads(out.stdout.strip().splitlines()[-1])
    if key == "GOAT_LAP_LISTS":
        assert listed == 0
    else:
        assert listed == st.list_bids
    if key == "GOAT_LAP_SKIP_IDLE":
        print(f"  phases passed over: {st.skipped_phases} (with the switch off: {skipped})")
        assert skipped == 0
        if kind == "nearperm":
            # a near-permutation leaves every later phase idle
            assert st.skipped_phases > 0
    else:
        assert skipped == st.skipped_phases
    assert (rounds, tail, phases) == (st.rounds, st.tail_bids, st.phases)
    assert np.array_equal(np.load(tmp_path / "p.npy").astype(np.int64), perm)


def test_lap_device_degenerate(G):
    perm, _ = G.lap_device(torch.full((1, 1), 3.0, device="cuda"))
    assert perm.cpu().tolist() == [0]
    perm, _ = G.lap_device(torch.full((50, 50), 0.25, device="cuda"))
    assert np.array_equal(perm.cpu().numpy(), np.arange(50))
    perm, _ = G.lap_device(torch.zeros((9, 9), device="cuda"))
    assert np.array_equal(perm.cpu().numpy(), np.arange(9))


def test_lap_device_rejects_nonfinite_and_round_cap(G):
    M = torch.rand((40, 40), device="cuda")
    M[3, 5] = float("nan")
    with pytest.raises(G.GoatError) as e:
        G.lap_device(M)
    assert e.value.status == G.GOAT_EINVAL
    M = torch.as_tensor(_scores("uniform", 300, 5), device="cuda")
    with pytest.raises(G.GoatError) as e:
        G.lap_device(M, max_rounds=4)
    assert e.value.status == G.GOAT_ENOTSUP
    # the library is usable after the refusal
    _check(G, _scores("uniform", 300, 5))


def test_solve_with_device_assignment(G):
    g = I.rho_sbm_pair([100, 100, 100], [[0.2, 0.01, 0.01], [0.01, 0.1, 0.01], [0.01, 0.01, 0.2]], 0.9, 9300)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    r1 = G.solve(A, B, return_P=True, lap=1)
    r0 = G.solve(A, B, lap=0)
    assert r1.stats.lap_device == 1 and r0.stats.lap_device == 0
    P = r1.P.cpu().numpy().astype(np.float64)
    c, _ = O.quantised_scores(P)
    _, best = O.lap_quantised(P)
    assert int(c[np.arange(300), r1.perm].sum()) == best
    # both projections score the same on P up to the quantisation bound
    _, s = O.quantised_scores(P)
    v1 = P[np.arange(300), r1.perm].sum()
    v0 = P[np.arange(300), r0.perm].sum()
    assert abs(v1 - v0) <= 300 * 2.0 ** -s
    print(f"match ratio device {O.match_ratio(r1.perm, g.truth):.4f}, host {O.match_ratio(r0.perm, g.truth):.4f}, "
          f"assignment ms device {r1.stats.ms_lap:.1f}, host {r0.stats.ms_lap:.1f}")


def test_run_steps_refused_after_device_assignment(G):
    # the device assignment takes G_Q and the packed operands as workspace
    g = I.rho_sbm_pair([60, 60], [[0.2, 0.02], [0.02, 0.2]], 0.9, 77)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    run = G.Run(A, B, prec="bf16x2", stop_on_stall=0, lap=1)
    run.steps(2)
    first = run.finish()
    with pytest.raises(G.GoatError) as e:
        run.steps(1)
    assert e.value.status == G.GOAT_EINVAL
    again = run.finish()
    run.close()
    assert np.array_equal(first.perm, again.perm)


def test_lap_device_planted_full_size(G):
    n = 10000
    gen = torch.Generator(device="cuda").manual_seed(12)
    M = torch.rand((n, n), generator=gen, device="cuda") * (1e-3 / n)
    truth = torch.randperm(n, generator=gen, device="cuda")
    M[torch.arange(n, device="cuda"), truth] += 0.9
    perm, st = G.lap_device(M)
    assert torch.equal(perm.long(), truth)
    print(f"n=10000 planted: rounds {st.rounds}, tail bids {st.tail_bids}, phases {st.phases}")


def test_lap_device_on_smooth_iterate_matches_host_optimum(G):
    # the assignment the solver makes at the end of a short run on the
    # weighted SBM workload (n = 4000): a smooth, nearly uniform P
    n = 4000
    g = I.weighted_sbm_pair([1000] * 4, [[0.02 if i == j else 0.005 for j in range(4)] for i in range(4)], 0.1,
                            4242)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    run = G.Run(A, B, prec="fp32", stop_on_stall=0, sk_max=300, lap=1)
    run.steps(4)
    P = run.finish(return_P=True).P
    run.close()
    perm, st = G.lap_device(P)
    pd = perm.cpu().numpy().astype(np.int64)
    Ph = P.double().cpu().numpy()
    from scipy.optimize import linear_sum_assignment
    ph = linear_sum_assignment(Ph, maximize=True)[1].astype(np.int64)   # independent reference
    rows = np.arange(n)
    vd, vh = Ph[rows, pd].sum(), Ph[rows, ph].sum()
    print(f"smooth iterate n={n}: device {vd:.9f} ({st.rounds} rounds, {st.tail_bids} sequential bids), "
          f"scipy {vh:.9f}")
    assert np.array_equal(np.sort(pd), rows)
    assert abs(vd - vh) <= n * 2.0 ** -st.shift
