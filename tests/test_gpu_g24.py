"""The 24-bit copy of the gradient read by the Sinkhorn sweeps
(goat_options.sk_g24): with the mixed products, the solver's per-iteration
step scalars stay within the mixed form's error band around the FP64
oracle, at fixed Sinkhorn sweep counts and with the tolerance stop.

The copy stores q = rint(G (2^23 - 1) / max|G|): each G_ij / eps a sweep
uses is within max|G| / eps 2^-24 = 2e-6 (natural units, at
eps = 0.03 max|G|) of its float value. An unconverged Sinkhorn iterate can
amplify a fixed perturbation of G (its slow modes), so the bound is the one
of the mixed products themselves: measured relative errors of fP, fQ and c
up to 4.7e-5 with the float G (bf16 hi/lo products, weighted pair,
n = 1000, three FW iterations) and 1.5e-5 with the 24-bit copy; bound
1e-4 for both."""
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


def _pair(kind, n):
    if kind == "wsbm":
        k = 4
        sizes = [n // k + (1 if r < n % k else 0) for r in range(k)]
        bp = np.full((k, k), 0.02); np.fill_diagonal(bp, 0.08)
        return I.weighted_sbm_pair(sizes, bp, 0.1, 4100 + n)
    return I.rho_er_pair(n, 0.05, 0.8, 4200 + n)


@pytest.mark.parametrize("prec,kind,n", [("bf16x3", "wsbm", 1000), ("bf16x2", "er", 1500), ("fp8", "er", 4500)])
def test_g24_matches_oracle_and_float_form(G, prec, kind, n):
    print(f"g24 prec={prec} kind={kind} n={n}", flush=True)
    g = _pair(kind, n)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    hist = {}
    for g24 in (0, 1):
        run = G.Run(A, B, prec=prec, sk_g24=g24, sk_max=40, sk_tol=0.0, stop_on_stall=0)
        run.steps(3)
        hist[g24] = run.history
        run.close()
    ref = O.goat(g.A, g.B, opt=O.GoatOptions(sk_max=40, sk_tol=0.0, fw_max=3, stop_on_stall=False), record=True)
    for k in range(3):
        h24, h32, o = hist[1][k], hist[0][k], ref.history[k]
        print(f"  it {k + 1}: fP {h24['fP']:.9g} / {h32['fP']:.9g} / oracle {o['fP']:.9g}; "
              f"c {h24['c']:.9g} / {o['c']:.9g}; t {h24['t']:.6f} / {o['t']:.6f}")
        assert h24["sk_iters"] == h32["sk_iters"] == o["sk_iters"] == 40
        for key in ("fP", "fQ", "c"):
            e24, e32 = abs(h24[key] - o[key]) / abs(o[key]), abs(h32[key] - o[key]) / abs(o[key])
            print(f"    {key}: 24-bit {e24:.2e}, float {e32:.2e}")
            assert e24 <= 1e-4 and e32 <= 1e-4, key
        assert h24["t"] == pytest.approx(o["t"], abs=1e-4)


def test_g24_tolerance_stop(G):
    # a converging solve stops on the same rule; sweeps within one of the
    # float form (the stored G differs from it by the rounding above)
    g = _pair("er", 1500)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    out = {}
    for g24 in (0, 1):
        r = G.solve(A, B, prec="bf16x2", sk_g24=g24, sk_max=1000, fw_max=4)
        out[g24] = r
    its = {k: [h["sk_iters"] for h in v.history] for k, v in out.items()}
    errs = [h["sk_err"] for h in out[1].history]
    print(f"sweeps float {its[0]}, 24-bit {its[1]}; 24-bit errors {errs}")
    assert len(its[0]) == len(its[1])
    for a, b in zip(its[0], its[1]):
        assert abs(a - b) <= 1
    for h in out[1].history:
        assert h["sk_iters"] >= 1000 or h["sk_err"] <= 1e-6
    # the final P differ at the solve's tolerance, so near-tied rows of the
    # assignment may go either way; the matchings agree as a whole
    mr = [float(np.mean(out[k].perm == g.truth)) for k in (0, 1)]
    print(f"match ratio float {mr[0]:.4f}, 24-bit {mr[1]:.4f}")
    assert abs(mr[0] - mr[1]) <= 0.005


def test_g24_refused_without_mixed_precision(G):
    g = _pair("er", 200)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    with pytest.raises(G.GoatError) as e:
        G.solve(A, B, prec="fp32", sk_g24=1)
    assert e.value.status == G.GOAT_EINVAL and "sk_g24" in str(e.value)
