"""Final assignment on the device (goat_lap_device) against the host solver
(goat_lap_max) on two n x n score matrices:

  iterate : P after `--fw` plain FP32 Frank-Wolfe iterations on the weighted
            4-block SBM pair (the benchmark's workload) — a smooth, nearly
            uniform P on which the assignment is hard for every solver;
  planted : 0.9 on a seeded permutation plus U(0, 1e-3/n) elsewhere.

Reported per matrix: device time (wall, host-synchronous call), parallel
rounds, sequential bids, phases, and — unless --no-host — the host time and
both objectives sum_i M[i, perm i] in float64 (the device is exact on the
quantised scores, within n 2^-s on M). One JSON line per matrix.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--fw", type=int, default=10)
    ap.add_argument("--no-host", action="store_true")
    ap.add_argument("--cases", default="planted,iterate")
    a = ap.parse_args(argv)

    import numpy as np
    import torch
    from paper_2111_05366_amd import goat, inputs

    t0 = time.perf_counter()

    def log(msg):
        print(f"[lap {time.perf_counter() - t0:6.1f}s] {msg}", file=sys.stderr, flush=True)

    goat.lib()
    n = a.n
    pair = inputs.workload_weighted_sbm(n)
    for case in a.cases.split(","):
        if case == "iterate":
            A = torch.as_tensor(pair.A, device="cuda")
            B = torch.as_tensor(pair.B, device="cuda")
            run = goat.Run(A, B, prec="fp32", stop_on_stall=0, sk_max=1000, lap=1)
            run.steps(a.fw)
            M = run.finish(return_P=True).P
            run.close()
            del A, B
            truth = pair.truth
        elif case == "planted":
            gen = torch.Generator(device="cuda").manual_seed(20211105)
            M = torch.rand((n, n), generator=gen, device="cuda") * (1e-3 / n)
            tp = torch.randperm(n, generator=gen, device="cuda")
            M[torch.arange(n, device="cuda"), tp] += 0.9
            truth = tp.cpu().numpy()
        else:
            raise ValueError(case)
        torch.cuda.synchronize()
        log(f"{case}: matrix ready")
        ts = time.perf_counter()
        perm, st = goat.lap_device(M)
        torch.cuda.synchronize()
        t_dev = time.perf_counter() - ts
        pd = perm.cpu().numpy().astype(np.int64)
        log(f"{case}: device {t_dev * 1e3:.1f} ms, {st.rounds} rounds, {st.tail_bids} sequential bids")
        out = dict(case=case, n=n, device_ms=round(t_dev * 1e3, 2), rounds=int(st.rounds),
                   sequential_bids=int(st.tail_bids), phases=int(st.phases), resolution_bits=int(st.resolution_bits),
                   match_ratio_device=float(np.mean(pd == truth)))
        if not a.no_host:
            Mh = M.double().cpu().numpy()
            ts = time.perf_counter()
            ph = goat.lap_max(Mh).astype(np.int64)
            t_host = time.perf_counter() - ts
            rows = np.arange(n)
            out.update(host_ms=round(t_host * 1e3, 1), value_device=float(Mh[rows, pd].sum()),
                       value_host=float(Mh[rows, ph].sum()), bound=float(n * 2.0 ** -st.shift),
                       match_ratio_host=float(np.mean(ph == truth)),
                       speedup=round(t_host / t_dev, 2))
            log(f"{case}: host {t_host * 1e3:.0f} ms")
        print(json.dumps(out), flush=True)
        del M


if __name__ == "__main__":
    main()
