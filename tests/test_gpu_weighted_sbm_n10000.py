"""End-to-end parity on the benchmark's workload, the weighted 4-block SBM
pair at n = 10,000, against the FP64 oracle's first three Frank-Wolfe
iterations (tests/golden/weighted_sbm_n10000_<form>.npz, written by
tests/golden/make_weighted_sbm_n10000.py, which calls only oracle/ and the
seeded input module). The two forms the benchmark times:

  plain : fp32 gradient, cold Sinkhorn start, float G in the sweeps;
  mixed : bf16 hi/lo gradient (three products), the warm-start network on
          the first iteration and the previous potentials afterwards (the
          oracle evaluates the same stored network in float64).

Replay: each device iteration runs the oracle's number of Sinkhorn sweeps
(goat_run_set_sinkhorn with tolerance 0), so both sides execute the same
steps and differ only by arithmetic. The tolerance-driven stop is compared
too, on the device's own sweep counts.

Bounds. Iterations 1 and 2 evaluate eps, fP and c at states both sides
share closely (the barycenter, then the first plan, whose solve takes 7
sweeps): the objective tolerance, 1e-5 relative (eps carries the gradient's
error at its largest entry, updated by linearity in FP32). fQ, and every
scalar from iteration 3 on, depend on a plan of a slow solve (972 sweeps at
iteration 2), which magnifies FP32 rounding of G along its slow modes: the
Q tolerance of 1e-4 relative then bounds eps and c (linear in the plan) by
1e-4 and f (quadratic) by 2e-4. Measured: 2e-8 to 5e-8 at the shared states
against 1.8e-5 to 2.4e-5 for the plan-level ones. The first plan's eight
stored rows: 1e-4 per entry. t: 1e-4 absolute.
Mixed form: its gradient differs from the FP64 one by the bf16 hi/lo split
(measured 6e-6 relative, bounded by 2e-5), which enters eps, fP and c at
first order (bounds 3e-5) and every plan entry through exp(G / eps) with
G / eps up to 1 / 0.03 = 33, so by up to 33 * 2e-5 = 7e-4 (bound 1e-3 per
entry; plan-level scalars 1e-3 for eps and c, 2e-3 for f).

The whole plain run to its stall is compared with the oracle's stored run
(weighted_sbm_n10000_plain_run.json, same script) iteration by iteration,
and the final match ratios against the benchmark's gate (0.005). From the
third iteration on, P is a capped 1000-sweep plan at eps near 0.03 max|G|
whose optimal assignment is decided below float resolution: the planted
permutation's objective <P, X> lies within 1.3e-7 relative of the optimum,
and a 1e-7 relative perturbation of P changes about half of the assigned
rows (measured after 3, 5 and 7 iterations: 49 %, 76 %, 76 %; at 1e-6,
79 % to 89 %). An fp32 gradient carries about 1e-6 relative rounding, so
its run cannot reproduce the FP64 run's assignment, only its scalars.
Where the match ratios differ by more than the gate, the test asserts that
reading instead: the device assignment is optimal for its own P within the
assignment's stated bound, the planted permutation is within 1e-6 relative
of that optimum, and a 1e-7 perturbation moves more than 10 % of the rows."""
import math
import os

import numpy as np
import pytest

from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
N = 10000

BOUNDS = {
    "plain": dict(eps=1e-5, state=1e-5, plan_c=1e-4, plan_f=2e-4, t=1e-4, q=1e-4),
    "mixed": dict(eps=3e-5, state=3e-5, plan_c=1e-3, plan_f=2e-3, t=1e-4, q=1e-3),
}


def _golden(form):
    path = os.path.join(HERE, "golden", f"weighted_sbm_n10000_{form}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} has not been generated")
    return np.load(path, allow_pickle=False)


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


@pytest.fixture(scope="module")
def pair(G):
    g = I.workload_weighted_sbm(N)
    return torch.as_tensor(g.A, device="cuda"), torch.as_tensor(g.B, device="cuda")


def _run(G, pair, form, **kw):
    from paper_2111_05366_amd import warmstart
    A, B = pair
    if form == "plain":
        return G.Run(A, B, prec="fp32", warm=0, stop_on_stall=0, sk_max=1000, sk_tol=1e-6, **kw)
    return G.Run(A, B, prec="bf16x3", warm=3, mlp_params=warmstart.load(), stop_on_stall=0,
                 sk_max=1000, sk_tol=1e-6, **kw)


def _rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("form", ["plain", "mixed"])
def test_replay_matches_oracle(G, pair, form):
    ref = _golden(form)
    bd = BOUNDS[form]
    run = _run(G, pair, form)
    rows = ref["rows"]
    for k in range(3):
        run.set_sinkhorn(int(ref["sk_iters"][k]), 0.0)
        assert run.steps(1) == 1
        h = run.history[-1]
        errs = {key: _rel(h[key], float(ref[key][k])) for key in ("eps", "fP", "fQ", "c")}
        print(f"{form} it {k + 1}: sweeps {h['sk_iters']} (oracle {int(ref['sk_iters'][k])}), "
              + ", ".join(f"{key} {v:.2e}" for key, v in errs.items())
              + f", t {h['t']:.6f} vs {float(ref['t'][k]):.6f}, sk_err {h['sk_err']:.2e} vs {float(ref['sk_err'][k]):.2e}",
              flush=True)
        assert h["sk_iters"] == int(ref["sk_iters"][k])
        assert errs["fQ"] <= bd["plan_f"]
        if k < 2:
            assert errs["eps"] <= bd["eps"]
            assert errs["fP"] <= bd["state"] and errs["c"] <= bd["state"]
        else:
            assert errs["eps"] <= bd["plan_c"]
            assert errs["fP"] <= bd["plan_f"] and errs["c"] <= bd["plan_c"]
        assert abs(h["t"] - float(ref["t"][k])) <= bd["t"]
        if k == 0:
            Q = run.direction()[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
            Qr = ref["Q_rows_it1"]
            m = Qr >= 1e-30
            qerr = float(np.max(np.abs(Q[m] - Qr[m]) / Qr[m]))
            fro = float(np.linalg.norm(Q - Qr) / np.linalg.norm(Qr))
            print(f"{form} it 1: Q rows element-wise {qerr:.2e}, Frobenius {fro:.2e}", flush=True)
            assert qerr <= bd["q"]
    run.close()


@pytest.mark.parametrize("form", ["plain", "mixed"])
def test_tolerance_stop_against_oracle(G, pair, form):
    # the device's own stop rule on the same pair: the sweep counts may
    # differ where a solve crosses the tolerance slowly (the FP32 marginal
    # error differs from the FP64 one by up to its compensated floor), and
    # both then stop within the tolerance band; the steps agree as in replay
    ref = _golden(form)
    run = _run(G, pair, form)
    run.steps(3)
    for k, h in enumerate(run.history):
        print(f"{form} free it {k + 1}: sweeps {h['sk_iters']} vs {int(ref['sk_iters'][k])}, "
              f"fP {_rel(h['fP'], float(ref['fP'][k])):.2e}, c {_rel(h['c'], float(ref['c'][k])):.2e}, "
              f"fQ {_rel(h['fQ'], float(ref['fQ'][k])):.2e}, t {h['t']:.6f} vs {float(ref['t'][k]):.6f}, "
              f"sk_err {h['sk_err']:.2e} vs {float(ref['sk_err'][k]):.2e}", flush=True)
        if int(ref["sk_iters"][k]) < 1000:
            assert h["sk_iters"] < 1000 and h["sk_err"] <= 1e-6
            assert abs(h["sk_iters"] - int(ref["sk_iters"][k])) <= 0.01 * int(ref["sk_iters"][k]) + 1
        else:
            assert h["sk_iters"] == 1000
        assert abs(h["t"] - float(ref["t"][k])) <= 1e-4
    run.close()


def test_plain_run_tracks_oracle(G, pair):
    # the whole plain run (tolerance stop, stop at the first zero step)
    # against the oracle's stored run of the same form
    # (weighted_sbm_n10000_plain_run.json); every iteration from the third on
    # evaluates plan-level quantities of capped 1000-sweep solves, so the
    # replay test's plan-level bounds apply (1e-4 for eps and c, 2e-4 for
    # fP and fQ), and each step t within 1e-4 where the step is resolved.
    # Near the stall the line search's linear coefficient b (the gain of
    # the full step) falls to 1e-7 |f|, below what the fp32 plans resolve
    # (device against oracle b: 34.335 / 34.302 at iteration 7, 0.0129 /
    # 0.0090 at iteration 8), so whether such a step is taken or is the
    # stall is decided by rounding: a step is resolved when the oracle's
    # |b| exceeds 1e-6 |fP|, and past the end of the shorter run every
    # step of the longer one, and the stall that ended the shorter run,
    # must be unresolved. The final assignments' match ratios agree within
    # 0.005, or the assignment is shown to be undetermined at float
    # resolution (module docstring). While the oracle run is still going
    # (it writes every iteration as it ends), the device's run is compared
    # with the iterations stored so far, and its final match ratio with
    # the oracle's after the same number of iterations.
    import json
    path = os.path.join(HERE, "golden", "weighted_sbm_n10000_plain_run.json")
    try:
        with open(path, encoding="utf-8") as fh:
            ref = json.load(fh)
    except (OSError, ValueError):
        pytest.skip("no readable stored oracle run")
    complete = bool(ref.get("complete"))
    if not ref.get("iterations"):
        pytest.skip("the stored oracle run has no iterations yet")
    g = I.workload_weighted_sbm(N)
    A, B = pair
    run = G.Run(A, B, prec="fp32", warm=0, stop_on_stall=1, sk_max=1000, sk_tol=1e-6, fw_max=30, lap=1)
    while run.steps(1) == 1:
        pass
    res = run.finish(return_P=True)
    run.close()
    its = ref["iterations"]
    print(f"plain run: {len(res.history)} FW iterations (oracle {len(its)})", flush=True)
    for k, (h, o) in enumerate(zip(res.history, its)):
        errs = {key: _rel(h[key], o[key]) for key in ("eps", "fP", "fQ", "c")}
        print(f"  it {k + 1}: sweeps {h['sk_iters']} / {int(o['sk_iters'])}, "
              + ", ".join(f"{key} {v:.2e}" for key, v in errs.items())
              + f", t {h['t']:.6f} / {o['t']:.6f}", flush=True)
        if int(o["sk_iters"]) < 1000:
            assert abs(h["sk_iters"] - int(o["sk_iters"])) <= 0.01 * int(o["sk_iters"]) + 1
        else:
            assert h["sk_iters"] == 1000
        bd = 1e-5 if k < 2 else 1e-4
        assert errs["eps"] <= bd and errs["c"] <= bd
        assert errs["fP"] <= 2 * bd and errs["fQ"] <= 2 * bd
        if abs(o["b"]) > 1e-6 * abs(o["fP"]):
            assert abs(h["t"] - o["t"]) <= 1e-4
    kd, ko = len(res.history), len(its)
    if kd < ko or (complete and kd > ko):
        longer = res.history if kd > ko else its
        for h in longer[min(kd, ko) - 1:]:
            assert abs(h["b"]) <= 1e-6 * abs(h["fP"])
    mr = float(np.mean(res.perm == g.truth))
    if complete:
        mr_ref = ref["match_ratio"]
    else:
        after = ref.get("match_ratio_after", {})
        if not after:
            return
        mr_ref = after.get(str(kd), after[max(after, key=int)])
    print(f"match ratio {mr:.4f} (oracle {mr_ref:.4f}{'' if complete else ', run in progress'})", flush=True)
    assert sorted(res.perm.tolist()) == list(range(N))
    if abs(mr - mr_ref) <= 0.005:
        return
    P = res.P
    rows = torch.arange(N, device=P.device)
    perm = torch.as_tensor(res.perm, device=P.device)
    P64 = P.double()

    def objective(p):
        return float(P64[rows, p.long()].sum())

    # the device assignment's bound on P itself: n 2^-s, s = R - 1 - e with
    # 2^(e-1) <= max P < 2^e and R = min(40, 55 - ceil(log2(n + 1)))
    e = math.frexp(float(P.max()))[1]
    s = min(40, 55 - math.ceil(math.log2(N + 1))) - 1 - e
    opt = objective(perm)
    planted = objective(torch.as_tensor(g.truth, device=P.device))
    gen = torch.Generator(device=P.device)
    gen.manual_seed(7)
    Pp = (P * (1 + 1e-7 * (2 * torch.rand((N, N), device=P.device, generator=gen) - 1))).contiguous()
    perm2, _ = G.lap_device(Pp)
    moved = float((perm2.long() != perm.long()).float().mean())
    print(f"assignment objective {opt:.9e}, planted {planted:.9e} ({planted / opt - 1:+.2e}); "
          f"rows moved by a 1e-7 perturbation: {moved:.3f}", flush=True)
    assert opt >= planted - N * 2.0 ** -s
    assert planted >= opt * (1 - 1e-6)
    assert moved > 0.10
