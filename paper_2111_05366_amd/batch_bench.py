"""Throughput of the batched solver on the random-start batch: 512
correlated ER pairs (n uniform in [50, 400], p in [0.05, 0.3], rho in
[0.6, 1.0]), 8 random doubly stochastic starts each, fp32, eps_rel = 0.03,
Sinkhorn tolerance 1e-6 (cap 1000), at most 30 FW iterations per start.

The shapes are autotuned first (goat_tune); then `--warmup` untimed and
`--launches` timed graph launches of the whole batch, each followed by the
final assignments and the choice among starts. Prints one JSON line:
FW iterations per second summed over all problems of the batch (device time
of the graph launch), problems per second, the final-assignment time, and
the mean match ratio of the kept permutations.
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
    ap.add_argument("--pairs", type=int, default=512)
    ap.add_argument("--restarts", type=int, default=8)
    ap.add_argument("--n-lo", type=int, default=50)
    ap.add_argument("--n-hi", type=int, default=400)
    ap.add_argument("--launches", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sk-max", type=int, default=1000)
    ap.add_argument("--fw-max", type=int, default=30)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--lap", type=int, default=0, choices=(0, 1),
                    help="final assignments: 0 host, 1 device")
    ap.add_argument("--warm", type=int, default=0, choices=(0, 1),
                    help="Sinkhorn start: 0 cold, 1 the previous FW iteration's column potentials")
    ap.add_argument("--cpu-sample", type=int, default=2, help="problems timed with the oracle (0: skip)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch
    from paper_2111_05366_amd import goat, inputs

    t0 = time.perf_counter()

    def log(msg):
        print(f"[batch {time.perf_counter() - t0:6.1f}s] {msg}", file=sys.stderr, flush=True)

    goat.lib()
    batch = inputs.workload_batch(a.pairs, a.restarts, a.n_lo, a.n_hi)
    log(f"generated {a.pairs} pairs x {a.restarts} starts")
    if not a.no_tune:
        goat.tune(a.n_hi, reps=2)
        shapes = {n: goat.tune_get(n) for n in (64, 128, 256, 400) if n <= a.n_hi}
        log(f"tuned shapes (lanes per row, waves): {shapes}")
    dev = [(torch.as_tensor(g.A, device="cuda"), torch.as_tensor(g.B, device="cuda"),
            torch.as_tensor(U, device="cuda")) for (g, U) in batch]
    b = goat.Batch(dev, restarts=a.restarts, sk_max=a.sk_max, fw_max=a.fw_max, sk_tol=1e-6, eps_rel=0.03,
                   warm=a.warm, lap=a.lap)
    log("batch created (graph captured)")
    for _ in range(a.warmup):
        b.launch()
        b.results()
    log("warmup done")
    graph_ms, lap_ms, fw_total, sk_total, capped = 0.0, 0.0, 0, 0, 0
    res = None
    for k in range(a.launches):
        b.launch()
        res = b.results()
        st = res["stats"]
        graph_ms += st.ms_graph
        lap_ms += st.ms_lap
        fw_total += st.fw_iters_total
        sk_total += st.sk_iters_total
        capped += st.sk_capped
        log(f"launch {k}: graph {st.ms_graph:.1f} ms, assignments {st.ms_lap:.1f} ms, FW iterations "
            f"{st.fw_iters_total}, Sinkhorn iterations {st.sk_iters_total}")
    mr = float(np.mean([np.mean(res["perm"][k] == g.truth) for k, (g, _) in enumerate(batch)]))
    nprob = a.pairs * a.restarts
    cpu = None
    if a.cpu_sample > 0:
        from oracle import goat_oracle as O
        hist = res["history"]
        done = 0
        t_orc = 0.0
        fw_orc = 0
        log("oracle sample ...")
        smallest = sorted(range(a.pairs), key=lambda k: batch[k][0].A.shape[0])
        for k in smallest[:a.cpu_sample]:
            g, U = batch[k]
            n = g.A.shape[0]
            P0 = O.random_init(U[:n].astype(np.float64))
            ts = time.perf_counter()
            r = O.goat(g.A, g.B, P0=P0, opt=O.GoatOptions(sk_max=a.sk_max, fw_max=a.fw_max))
            t_orc += time.perf_counter() - ts
            fw_orc += r.fw_iters
            done += 1
        cpu = dict(value=fw_orc / t_orc, unit="FW iters/s", cores=1, kind="oracle",
                   sample=f"the {done} smallest problems of the batch (start 0), {fw_orc} FW iterations "
                          f"in {t_orc:.1f} s")
        del hist
    line = dict(
        metric="batched GOAT FW iterations/s (all problems of the batch, device time)",
        value=round(fw_total / (graph_ms * 1e-3), 1), unit="FW iters/s",
        problems_per_s=round(a.launches * nprob / (graph_ms * 1e-3), 1),
        ms_graph_per_launch=round(graph_ms / a.launches, 2), ms_assign_per_launch=round(lap_ms / a.launches, 2),
        fw_iters_per_launch=fw_total // a.launches, sk_iters_per_launch=sk_total // a.launches,
        sk_capped_per_launch=capped // a.launches, kernels_in_graph=res["stats"].launches,
        match_ratio_mean=round(mr, 4), dtype="f32+f64", data="synthetic",
        config=dict(workload=f"{a.pairs} correlated ER pairs, n in [{a.n_lo},{a.n_hi}], p in [0.05,0.3], "
                             f"rho in [0.6,1.0], {a.restarts} random starts each",
                    sk_max=a.sk_max, fw_max=a.fw_max, sk_tol=1e-6, eps_rel=0.03, warm=a.warm, lap=a.lap),
        cpu_baseline=cpu)
    b.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
