"""LOT against the exact assignment on Uniform(100, 150) costs (the paper's
LOT-versus-LAP comparison): the entropic plan's objective and its rounded
permutation stay within 0.5 % of the optimal assignment."""
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


@pytest.mark.parametrize("n", [250, 1000])
def test_lot_within_half_percent_of_lap(G, n):
    from scipy.optimize import linear_sum_assignment
    for r in range(2):
        M = I.cost_matrix(n, 1000 * n + r).astype(np.float64)
        # exact assignment: the oracle's Hungarian method at n = 250, SciPy's
        # solver at n = 1000 (the plain Python loop would take minutes)
        perm = O.hungarian_max(-M) if n <= 250 else linear_sum_assignment(M)[1]
        ofv_lap = float(M[np.arange(n), perm].sum())
        out = G.sinkhorn(torch.as_tensor(-M.astype(np.float32), device="cuda"), eps=0.01, max_iter=5000, tol=1e-4)
        Q = out.Q.double().cpu().numpy()
        gap_soft = (ofv_lap - float(np.sum(M * Q))) / ofv_lap
        pr = G.lap_max(Q)
        gap_round = (ofv_lap - float(M[np.arange(n), pr].sum())) / ofv_lap
        print(f"n={n} rep {r}: soft gap {gap_soft:.2e}, rounded gap {gap_round:.2e}, "
              f"iters {int(out.iters.item())}, err {float(out.err.item()):.1e}")
        # gap = (OFV_LAP - OFV_LOT) / OFV_LAP of a minimisation: a doubly
        # stochastic plan costs at least the optimal assignment, so gap <= 0
        # up to the plan's marginal slack. The device plan meets its row
        # marginals only to tol = 1e-4, which can lower <M, Q> below the
        # optimum by about tol * max M / mean M = 1e-4 * 150 / 125 = 1.2e-4 of
        # it (upper bound 1.5e-4). The paper's claim is a gap within 0.5 %.
        assert -5e-3 <= gap_soft <= 1.5e-4
        # a permutation cannot beat the optimum at all
        assert -5e-3 <= gap_round <= 1e-12
