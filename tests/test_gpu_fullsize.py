"""Parity at the benchmark's full size (n = 10,000, the launch
configuration bench.py times) on outputs the FP64 oracle can compute one by
one, and properties that hold at any size; plus element-wise Sinkhorn parity
at n = 4500, which runs the same 1024-thread strip configuration.

Inputs are seeded draws from paper_2111_05366_amd.inputs only."""
import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_FULL = 10000


@pytest.fixture(scope="module", autouse=True)
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


@pytest.fixture(scope="module")
def pair():
    return I.workload_weighted_sbm(N_FULL)


def _lse(x, axis):
    m = np.max(x, axis=axis, keepdims=True)
    return (m + np.log(np.sum(np.exp(x - m), axis=axis, keepdims=True))).squeeze(axis)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_gradient_sampled_entries_full_size(G, pair, prec):
    n = N_FULL
    P = I.uniform_matrix(n, 4242) / np.float32(n)
    A, B = pair.A, pair.B
    Gd = G.grad(torch.as_tensor(A, device="cuda"), torch.as_tensor(B, device="cuda"),
                torch.as_tensor(P, device="cuda"), prec=prec)
    got = Gd.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    rows = rng.choice(n, size=4, replace=False)
    cols = rng.choice(n, size=6, replace=False)
    Ad, Bd, Pd = A.astype(np.float64), B.astype(np.float64), P.astype(np.float64)
    # G_ij = (A P B^T)_ij + (A^T P B)_ij for the sampled rows, all columns
    ref_rows = (Ad[rows] @ Pd) @ Bd.T + (Ad.T[rows] @ Pd) @ Bd
    err = np.max(np.abs(got[rows] - ref_rows)) / np.max(np.abs(ref_rows))
    ref_cols = Ad @ (Pd @ Bd.T[:, cols]) + Ad.T @ (Pd @ Bd[:, cols])
    err_c = np.max(np.abs(got[:, cols] - ref_cols)) / np.max(np.abs(ref_cols))
    print(f"grad n={n} {prec}: sampled rows rel {err:.2e}, sampled cols rel {err_c:.2e}")
    assert err <= 1e-4 and err_c <= 1e-4


def test_gradient_general_pair_bf16x3_n4500(G):
    """A general (non-symmetric) pair at n = 4500 in the bf16 hi/lo form: the
    first product stacks [B; B^T] (rows 2 np) and runs on the fused
    three-segment eight-wave kernel, the second has six segments and runs
    segment by segment. Sampled rows and columns of G against FP64."""
    n = 4500
    A = I.random_matrix(n, n, 61, 0.0, 1.0)
    B = I.random_matrix(n, n, 62, 0.0, 1.0)
    P = I.uniform_matrix(n, 63) / np.float32(n)
    Gd = G.grad(torch.as_tensor(A, device="cuda"), torch.as_tensor(B, device="cuda"),
                torch.as_tensor(P, device="cuda"), prec="bf16x3", symmetric=False)
    got = Gd.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    rows = rng.choice(n, size=4, replace=False)
    cols = rng.choice(n, size=6, replace=False)
    Ad, Bd, Pd = A.astype(np.float64), B.astype(np.float64), P.astype(np.float64)
    ref_rows = (Ad[rows] @ Pd) @ Bd.T + (Ad.T[rows] @ Pd) @ Bd
    ref_cols = Ad @ (Pd @ Bd.T[:, cols]) + Ad.T @ (Pd @ Bd[:, cols])
    err = np.max(np.abs(got[rows] - ref_rows)) / np.max(np.abs(ref_rows))
    err_c = np.max(np.abs(got[:, cols] - ref_cols)) / np.max(np.abs(ref_cols))
    print(f"grad n={n} bf16x3 general: sampled rows rel {err:.2e}, sampled cols rel {err_c:.2e}")
    assert err <= 1e-4 and err_c <= 1e-4


def test_gradient_fp8_sampled_entries_er5000(G):
    """FP8 form on the 0/1 correlated ER pair at n = 5000 (p = 0.02,
    rho = 0.7): sampled rows and columns of G against FP64."""
    g = I.workload_er_5000()
    n = g.A.shape[0]
    P = I.uniform_matrix(n, 4343) / np.float32(n)
    Gd = G.grad(torch.as_tensor(g.A, device="cuda"), torch.as_tensor(g.B, device="cuda"),
                torch.as_tensor(P, device="cuda"), prec="fp8")
    got = Gd.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(8)
    rows = rng.choice(n, size=4, replace=False)
    cols = rng.choice(n, size=6, replace=False)
    Ad, Bd, Pd = g.A.astype(np.float64), g.B.astype(np.float64), P.astype(np.float64)
    ref_rows = 2.0 * (Ad[rows] @ Pd) @ Bd
    ref_cols = 2.0 * Ad @ (Pd @ Bd[:, cols])
    err = np.max(np.abs(got[rows] - ref_rows)) / np.max(np.abs(ref_rows))
    err_c = np.max(np.abs(got[:, cols] - ref_cols)) / np.max(np.abs(ref_cols))
    print(f"grad n={n} fp8: sampled rows rel {err:.2e}, sampled cols rel {err_c:.2e}")
    assert err <= 1e-4 and err_c <= 1e-4


def test_sinkhorn_first_iteration_full_size(G):
    """After one iteration from g = 0: f_i = -eps LSE_j(G_ij/eps) and
    g_j = -eps LSE_i((G_ij + f_i)/eps), all n of each, in FP64."""
    n = N_FULL
    Gm = I.random_matrix(n, n, 515, -1.0, 1.0)
    out = G.sinkhorn(torch.as_tensor(Gm, device="cuda"), eps_rel=0.03, max_iter=1, tol=0.0, want_Q=False)
    eps = float(out.eps.item())
    Gd = Gm.astype(np.float64) / eps
    f = -eps * _lse(Gd, 1)
    g = -eps * _lse(Gd + (f / eps)[:, None], 0)
    df = np.max(np.abs(out.f.cpu().numpy() - f)) / eps
    dg = np.max(np.abs(out.g.cpu().numpy() - g)) / eps
    print(f"sinkhorn n={n} first iteration: |df|/eps {df:.2e} |dg|/eps {dg:.2e}")
    assert df <= 1e-4 and dg <= 1e-4


def test_sinkhorn_marginals_full_size(G, pair):
    """Properties after 30 iterations on the workload's gradient at J:
    column sums of Q are 1 (the last update is a column update), and the
    reported error is the largest row-sum deviation of the returned Q."""
    n = N_FULL
    A = torch.as_tensor(pair.A, device="cuda")
    B = torch.as_tensor(pair.B, device="cuda")
    J = torch.full((n, n), 1.0 / n, device="cuda")
    Gd = G.grad(A, B, J, prec="fp32")
    out = G.sinkhorn(Gd, eps_rel=0.03, max_iter=30, tol=0.0)
    Q = out.Q.double()
    cols = (Q.sum(dim=0) - 1).abs().max().item()
    rows = (Q.sum(dim=1) - 1).abs().max().item()
    print(f"marginals n={n}: max col dev {cols:.2e}, max row dev {rows:.2e}, reported {out.err.item():.2e}")
    assert cols <= 2e-5
    assert abs(rows - float(out.err.item())) <= 1e-6 + 1e-3 * rows
    assert int(out.iters.item()) == 30


@pytest.mark.parametrize("iters", [1, 7])
def test_sinkhorn_parity_1024_thread_strips(G, iters):
    n = 4500
    Gm = I.random_matrix(n, n, 616, -1.0, 1.0)
    out = G.sinkhorn(torch.as_tensor(Gm, device="cuda"), eps_rel=0.03, max_iter=iters, tol=0.0)
    eps = float(out.eps.item())
    ref = O.log_sinkhorn_max(Gm.astype(np.float64), eps, tol=0.0, max_iter=iters)
    Q = out.Q.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(Q - ref.Q) / np.linalg.norm(ref.Q)
    dg = np.max(np.abs(out.g.cpu().numpy() - ref.g)) / eps
    print(f"sinkhorn n={n} iters={iters}: Q rel_fro {err:.2e}, |dg|/eps {dg:.2e}")
    assert int(out.iters.item()) == iters == ref.iters
    assert err <= 1e-4 and dg <= 1e-4
