#!/usr/bin/env python3
"""CAVI sweep throughput on one MI355X.

Workload (default ``c2``): one synthetic dataset of N=1,000,000 rows x G=96
genes with K=8 subpopulations, proportions ~ Dirichlet(0.5 1_8), means ~
U(15, 35), precisions ~ Gamma(2, rate 0.5), FP32 data generated on the GPU
and resident in HBM before timing.  A step is one full CAVI sweep (E-step,
log-sum-exp responsibilities, statistics, conjugate updates, lower bound,
convergence test).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "CAVI sweeps/s (N·K·G elems/s, %HBM peak); time-to-ELBO-conv plain vs batched+warm"
HBM_PEAK_GBS = 8000.0
DOMINANT_KERNEL = "k_estep_stats"
KERNEL_SRC = os.path.join(ROOT, "paper_2401_10068_amd", "csrc", "cavi_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None
    when they were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(x_host, K: int, seed: int, budget_s: float):
    """The FP64 oracle, as it stands, on the host: whole sweeps of the same workload."""
    from oracle import cavi_oracle as oc

    N, G = x_host.shape
    pr = oc.Prior()
    m0 = oc.data_mean(x_host)
    st = oc.init_standard(x_host, K, pr, m0, seed)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        oc.sweep(x_host, pr, m0, st)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {
        "value": N * K * G * sweeps / el,
        "unit": "N*K*G elems/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sweeps} full sweep(s) of the same {N}x{G}, K={K} dataset from the standard initial state "
                  f"({el:.1f} s, single-threaded FP64 C)",
    }


def batch_bench(args) -> int:
    """Time to ELBO convergence (1e-6 relative) of a batch of datasets: batched
    (one set of launches per sweep for all datasets) against plain GPU CAVI run
    one dataset at a time (on an evenly spaced sample of the datasets)."""
    import numpy as np
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.cavi import Cavi, CaviBatch

    Ns, Ks, rec, seed = synth.batch_workload(args.workload)
    G = rec.G
    x, row_off, _, _, _, _, _ = synth.make_batch_gpu(seed, Ns, Ks, rec)
    torch.cuda.synchronize()
    bt = CaviBatch(x, Ns, Ks)
    t0 = time.perf_counter()
    bt.init_standard(seed)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    sw, el, nconv = bt.run(args.max_sweeps, 1e-6)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    bt.close()
    nkg = float((sw.astype(np.float64) * Ns * Ks * G).sum())
    bytes_read = float((sw.astype(np.float64) * Ns * 4 * G).sum())
    # plain: one handle per dataset, standard initialisation, run to convergence
    idx = np.arange(0, Ns.size, max(1, Ns.size // args.plain_sample))
    t_plain = 0.0
    plain_sw = []
    max_rel = 0.0
    for b in idx:
        xb = x[int(row_off[b]):int(row_off[b + 1])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cx = Cavi(xb, int(Ks[b]))
        cx.init_standard(seed + int(b))
        n, L, conv = cx.run(args.max_sweeps, 1e-6)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        cx.close()
        plain_sw.append(n)
        max_rel = max(max_rel, abs(L - el[b]) / abs(el[b]))
    frac = float((Ns[idx] * Ks[idx]).sum() / (Ns * Ks).sum())
    out = {
        "metric": METRIC,
        "value": nkg / t_run,
        "unit": "N*K*G elems/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "f32",
        "config": {"workload": f"{Ns.size} datasets ({args.workload}): N log-uniform in [{Ns.min()}, {Ns.max()}], "
                               f"K in {{{Ks.min()}..{Ks.max()}}}, G={G}, seed {seed}, run to 1e-6"},
        "batched": {"init_s": t_init, "run_s": t_run, "converged": nconv, "datasets": int(Ns.size),
                    "sweeps_total": int(sw.sum()), "sweeps_median": float(np.median(sw)), "sweeps_max": int(sw.max()),
                    "effective_GBps": bytes_read / t_run / 1e9},
        "plain_one_at_a_time": {"sample": int(idx.size), "sample_s": t_plain,
                                "extrapolated_s": t_plain / frac, "sweeps_median": float(np.median(plain_sw)),
                                "max_rel_elbo_diff_vs_batched": max_rel},
        "speedup_batched_vs_plain": (t_plain / frac) / (t_init + t_run),
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=["small", "c2", "c3", "c4", "c5eval"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--max-sweeps", type=int, default=10000, help="batched workloads: sweep cap")
    ap.add_argument("--plain-sample", type=int, default=256, help="batched workloads: datasets timed one at a time")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sweep shards over rows with one "
              "all-reduce of the statistics per sweep, which this build does not run.", file=sys.stderr)
        return 2
    sys.path.insert(0, ROOT)
    if args.workload in ("c4", "c5eval"):
        return batch_bench(args)
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.cavi import Cavi

    N, rec, seed = synth.workload(args.workload)
    K, G = rec.K, rec.G
    x, _, _, _, _ = synth.make_dataset_gpu(seed, 0, N, rec)
    torch.cuda.synchronize()
    cx = Cavi(x, K)
    cx.init_standard(seed)
    if args.warmup:
        cx.sweep(args.warmup, want_elbo=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    elbo = cx.sweep(args.steps, want_elbo=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0

    est_ms = cx.profile_estep(20)
    bytes_per_sweep = 4.0 * N * G  # X read once per sweep, FP32
    achieved = bytes_per_sweep / (est_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    ms_per_step = sec / args.steps * 1e3
    nkg = float(N) * K * G
    out = {
        "metric": METRIC,
        "value": nkg * args.steps / sec,
        "unit": "N*K*G elems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"single dataset N={N} x G={G}, K={K} ({args.workload}), seed {seed}",
                   "N": N, "G": G, "K": K},
        "sweeps_per_s": args.steps / sec,
        "sweep_hbm_frac": bytes_per_sweep / (sec / args.steps) / 1e9 / HBM_PEAK_GBS,
        "elbo_last": float(elbo[-1]),
        "roofline": {
            "kernel": DOMINANT_KERNEL,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_ms": est_ms,
            "bytes_per_launch": bytes_per_sweep,
        },
    }
    cx.close()
    if not args.no_cpu:
        xh = x.cpu().numpy()
        del x
        out["cpu_baseline"] = cpu_baseline(xh, K, seed, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
