"""Short driver for hardware-counter passes (rocprofv3 --pmc).

Default (`--what sinkhorn`), on the weighted SBM workload at n = 10,000:

Steps, each printed as it ends: the gradient at a Frank-Wolfe iterate past
the first two (where Sinkhorn does not converge within the cap), a plain
device copy of n^2 floats (the calibration kernel: 4 n^2 bytes read and
4 n^2 written), then `--sweeps` Sinkhorn iterations in the plain form and
the same number in the compensated form. Nothing here is timed; byte
counters of the row sweep are read per dispatch and scaled by what the copy
kernel's counters read for its known traffic.

`--what sinkhorn24`: the same calibration copy, then the solver's mixed form
(bf16 hi/lo gradient, Sinkhorn on the 24-bit copy of G) for `--fw`
Frank-Wolfe iterations of `--sweeps` sweeps each (tolerance 0, so every
sweep is a full launch of the 24-bit row kernel).

`--what gemm`: gradient products only, each printed as it ends: the bf16
hi/lo gradient (3-segment products) and the fp32 gradient of the weighted
SBM pair at n = 10,000 at its barycenter, then the fp8 gradient of the
correlated ER pair at n = 5000 (p = 0.02, rho = 0.7), `--reps` times each.
For MFMA utilisation and LDS counters per dispatch.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--sweeps", type=int, default=8)
    ap.add_argument("--fw", type=int, default=2, help="FW iterations before the measured gradient")
    ap.add_argument("--what", choices=("sinkhorn", "sinkhorn24", "gemm"), default="sinkhorn")
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    if a.what == "gemm":
        return gemm_products(a)
    if a.what == "sinkhorn24":
        return sinkhorn24(a)

    import torch
    from paper_2111_05366_amd import goat, inputs

    t0 = time.perf_counter()

    def log(msg):
        print(f"[counters {time.perf_counter() - t0:6.1f}s] {msg}", flush=True)

    n = a.n
    pair = inputs.workload_weighted_sbm(n)
    A = torch.as_tensor(pair.A, device="cuda")
    B = torch.as_tensor(pair.B, device="cuda")
    run = goat.Run(A, B, prec="fp32", sk_max=200, stop_on_stall=0)
    run.steps(a.fw)
    G = run.gradient()
    run.close()
    torch.cuda.synchronize()
    log(f"gradient after {a.fw} FW iterations (n={n})")
    src = torch.ones((n, n), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy of {4 * n * n} bytes")
    del src, dst
    # tolerance 1e-5: plain sweeps (the form used far from the tolerance)
    out = goat.sinkhorn(G, max_iter=a.sweeps, tol=1e-5, want_Q=False)
    torch.cuda.synchronize()
    log(f"{a.sweeps} plain sweeps, err {float(out.err.item()):.2e}")
    out = goat.sinkhorn(G, max_iter=a.sweeps, tol=0.0, want_Q=False)
    torch.cuda.synchronize()
    log(f"{a.sweeps} compensated sweeps, err {float(out.err.item()):.2e}")


def sinkhorn24(a):
    import torch
    from paper_2111_05366_amd import goat, inputs

    t0 = time.perf_counter()

    def log(msg):
        print(f"[counters {time.perf_counter() - t0:6.1f}s] {msg}", flush=True)

    n = a.n
    pair = inputs.workload_weighted_sbm(n)
    A = torch.as_tensor(pair.A, device="cuda")
    B = torch.as_tensor(pair.B, device="cuda")
    src = torch.ones((n, n), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy of {4 * n * n} bytes")
    del src, dst
    run = goat.Run(A, B, prec="bf16x3", sk_g24=1, sk_max=a.sweeps, sk_tol=0.0, stop_on_stall=0)
    for k in range(a.fw):
        run.steps(1)
        log(f"FW iteration {k + 1}: {a.sweeps} sweeps on the 24-bit copy of G")
    run.close()


def gemm_products(a):
    import torch
    from paper_2111_05366_amd import goat, inputs

    t0 = time.perf_counter()

    def log(msg):
        print(f"[counters {time.perf_counter() - t0:6.1f}s] {msg}", flush=True)

    n = a.n
    pair = inputs.workload_weighted_sbm(n)
    A = torch.as_tensor(pair.A, device="cuda")
    B = torch.as_tensor(pair.B, device="cuda")
    P = torch.full((n, n), 1.0 / n, device="cuda")
    for prec in ("bf16x3", "fp32"):
        for _ in range(a.reps):
            goat.grad(A, B, P, prec=prec)
        torch.cuda.synchronize()
        log(f"{a.reps} {prec} gradients at n={n}")
    del A, B, P
    g = inputs.workload_er_5000()
    m = g.A.shape[0]
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    P = torch.full((m, m), 1.0 / m, device="cuda")
    for _ in range(a.reps):
        goat.grad(A, B, P, prec="fp8")
    torch.cuda.synchronize()
    log(f"{a.reps} fp8 gradients at n={m}")
    goat.release_workspace()


if __name__ == "__main__":
    main()
