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
DOMINANT_KERNEL = "k_estep_tiled"
KERNEL_SRC = os.path.join(ROOT, "paper_2401_10068_amd", "csrc", "estep_tiled.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


LM_KERNEL = "k_lm_pass"  # the per-gene pass of the linear-mixing VB and EM
LM_SRC = os.path.join(ROOT, "paper_2401_10068_amd", "csrc", "linmix.h")
GIBBS_KERNEL = "k_gibbs_pass"
GIBBS_SRC = os.path.join(ROOT, "paper_2401_10068_amd", "csrc", "gibbs.hip")


def kernel_sha(src: str = KERNEL_SRC) -> str:
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, src: str = KERNEL_SRC):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None
    when they were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_sha(src):
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(x_host, K: int, seed: int, budget_s: float):
    """The FP64 oracle, as it stands, on the host: whole sweeps of the same workload from its
    standard initial state, first on one thread, then with its rows split over every core this
    process may use (per-thread FP64 sums added in thread order).  ``value`` is the all-core
    rate; the single-thread rate is reported beside it."""
    from oracle import cavi_oracle as oc

    N, G = x_host.shape
    pr = oc.Prior()
    m0 = oc.data_mean(x_host)
    st = oc.init_standard(x_host, K, pr, m0, seed)

    def timed(step, budget):
        n = 0
        t0 = time.perf_counter()
        while True:
            step()
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return n, el

    s1, e1 = timed(lambda: oc.sweep(x_host, pr, m0, st), budget_s / 2)
    used = [0]

    def mt():
        used[0] = oc.sweep_mt(x_host, pr, m0, st)[1]

    sm, em = timed(mt, budget_s / 2)
    return {
        "value": N * K * G * sm / em,
        "unit": "N*K*G elems/s",
        "cores": used[0],
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "single_thread": {"value": N * K * G * s1 / e1, "cores": 1, "sweeps": s1, "seconds": e1},
        "sample": f"{sm} full sweep(s) of the same {N}x{G}, K={K} dataset on {used[0]} threads ({em:.1f} s), "
                  f"after {s1} on one thread ({e1:.1f} s); FP64 C with OpenMP over rows, from the standard "
                  f"initial state",
    }


def copy_reference(device) -> dict:
    """Achievable HBM rates on this GPU, over 1.5 GB (far beyond the caches): a device-to-device
    copy (torch; bytes read + written, best of five, timed with events) and the library's plain
    streaming read (cavi_probe_read, 16-byte loads; the best of a few grid sizes)."""
    import torch

    from paper_2401_10068_amd.cavi import cavi_probe_read

    n = 384_000_000
    src = torch.ones(n, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    ts = []
    for _ in range(5):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    tc = min(ts)
    del dst
    out = torch.zeros(16384, dtype=torch.float32, device=device)
    reads = {}
    for grid in (1024, 2048, 4096, 8192, 16384):
        ms = cavi_probe_read(src, out, grid, 5)
        reads[grid] = 4 * n / (ms * 1e-3) / 1e9
    torch.cuda.synchronize()
    ok = abs(float(out[:16384].double().sum()) - n) <= 1e-6 * n  # every float read once
    del src, out
    best = max(reads, key=reads.get)
    return {"copy_GBps": 2 * 4 * n / tc / 1e9, "read_GBps": reads[best], "read_grid": best,
            "read_GBps_by_grid": {str(k): round(v, 1) for k, v in reads.items()}, "read_sum_ok": ok,
            "bytes": 4 * n}


def lm_bench(args) -> int:
    """The paper's own model (Section 3.3) and variational Bayes (eqs 16-31): V genes with N = 3
    networks, the weights K = (0.1, 0.3) of its first synthetic study (Section 4), rho = 100 and its
    precision matrix; random 0/1 expression profiles stand in for the Boolean-network outputs.
    A step is one sweep (q(rho), every q(beta_i), q(K, Lambda), the bound)."""
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.lmvb import LinMixVB

    V, N, K_true, seed = 10_000_000, 3, (0.1, 0.3), 2
    r, d = synth.linmix_dataset(seed, V, K_true)
    rd, dd = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    h = LinMixVB(rd, dd)
    h.init()
    if args.warmup:
        h.sweep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    elbo = h.sweep(args.steps)
    sec = time.perf_counter() - t0
    pass_ms = h.profile_pass(20)
    h.close()
    bytes_per_pass = 8.0 * V * (N + 1)  # r and d read once, FP64
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    # the paper's synthetic study (Section 4, Table 1): its five weight vectors, V = 8000 genes (its
    # largest data size), 100 iterations (its VB converged in 100); then the time to convergence
    table1 = []
    TABLE1 = [((0.1, 0.3), (0.1031, 0.2992)), ((0.13, 0.25), (0.1218, 0.2351)), ((0.39, 0.54), (0.3814, 0.5342)),
              ((0.25, 0.16), (0.2469, 0.1961)), ((0.18, 0.29), (0.1791, 0.2678))]
    for row, (k_true, k_paper) in enumerate(TABLE1):
        rs, ds = synth.linmix_dataset(1 + row, 8000, k_true)
        hs = LinMixVB(torch.from_numpy(rs).cuda(), torch.from_numpy(ds).cuda())
        hs.init()
        hs.sweep(100)
        ke = hs.globals()["K0K"]
        hs.close()
        table1.append({"actual": list(k_true), "vb": [round(float(v), 4) for v in ke],
                       "error": float(((ke[0] - k_true[0]) ** 2 + (ke[1] - k_true[1]) ** 2) ** 0.5),
                       "paper_vb": list(k_paper)})
    rs, ds = synth.linmix_dataset(1, 8000, (0.1, 0.3))
    hs = LinMixVB(torch.from_numpy(rs).cuda(), torch.from_numpy(ds).cuda())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs.init()
    n_conv, L_conv, conv = hs.run(10000, 1e-6)
    conv_s = time.perf_counter() - t0
    hs.close()
    if args.copy_ref:
        src = torch.ones(96_000_000, dtype=torch.float32, device=rd.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": "VB sweeps/s of the paper's linear-mixing model (genes x sweeps / s, %HBM peak)",
        "value": V * args.steps / sec,
        "unit": "genes*sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"linear-mixing VB (Section 3.3), V={V} genes, N={N}, K={K_true}, rho=100, seed {seed}",
                   "V": V, "N": N},
        "elbo_last": float(elbo[-1]),
        "roofline": {
            "kernel": LM_KERNEL,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("lm", LM_SRC),
            "avg_ms": pass_ms,
            "bytes_per_launch": bytes_per_pass,
        },
        "table1": table1,
        "table1_mean_error": sum(t["error"] for t in table1) / len(table1),
        "time_to_convergence_V8000": {"rel_tol": 1e-6, "seconds": conv_s, "sweeps": n_conv, "converged": conv,
                                      "elbo": L_conv},
    }
    if not args.no_cpu:
        from oracle import lmvb_oracle as lo

        Vs = 1_000_000
        pr = lo.default_prior(N)
        st = lo.init_state(Vs, pr)
        sweeps = 0
        t0 = time.perf_counter()
        while True:
            lo.sweep(r[:Vs], d[:Vs], st, pr)
            lo.elbo(r[:Vs], d[:Vs], st, pr)
            sweeps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": Vs * sweeps / el, "unit": "genes*sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} sweep(s) with the bound of the first {Vs} genes of the same data from the initial "
                      f"state ({el:.1f} s, numpy FP64, one thread)"}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


def em_bench(args) -> int:
    """The paper's expectation maximisation for its linear-mixing model (Section 4.2, eqs 42-47) on
    the same genes as the variational workload: V genes with N = 3 networks, K = (0.1, 0.3),
    rho = 100.  A step is one iteration (the E-step of every gene, the M-step, the log-likelihood of
    the estimates it started from and the stopping test)."""
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.lmem import LinMixEM

    V, N, K_true, seed = 10_000_000, 3, (0.1, 0.3), 2
    r, d = synth.linmix_dataset(seed, V, K_true)
    rd, dd = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    h = LinMixEM(rd, dd)
    if args.warmup:
        h.iterate(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ll = h.iterate(args.steps)
    sec = time.perf_counter() - t0
    pass_ms = h.profile_pass(20)
    h.close()
    bytes_per_pass = 8.0 * V * (N + 1)  # r and d read once, FP64
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    # the EM column of Table 1: its five weight vectors, V = 8000 genes, 100 iterations (its EM
    # converged in 100); then the time to convergence
    table1 = []
    TABLE1_EM = [((0.1, 0.3), (0.1013, 0.3013)), ((0.13, 0.25), (0.1218, 0.2341)), ((0.39, 0.54), (0.3812, 0.5341)),
                 ((0.25, 0.16), (0.2468, 0.1939)), ((0.18, 0.29), (0.1811, 0.2671))]
    for row, (k_true, k_paper) in enumerate(TABLE1_EM):
        rs, ds = synth.linmix_dataset(1 + row, 8000, k_true)
        hs = LinMixEM(torch.from_numpy(rs).cuda(), torch.from_numpy(ds).cuda())
        hs.iterate(100)
        ke = hs.params()["K"]
        hs.close()
        table1.append({"actual": list(k_true), "em": [round(float(v), 4) for v in ke],
                       "error": float(((ke[0] - k_true[0]) ** 2 + (ke[1] - k_true[1]) ** 2) ** 0.5),
                       "paper_em": list(k_paper)})
    rs, ds = synth.linmix_dataset(1, 8000, (0.1, 0.3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = LinMixEM(torch.from_numpy(rs).cuda(), torch.from_numpy(ds).cuda())
    n_conv, ll_conv, conv = hs.run(10000, 1e-7)
    conv_s = time.perf_counter() - t0
    hs.close()
    if args.copy_ref:
        src = torch.ones(96_000_000, dtype=torch.float32, device=rd.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": "EM iterations/s of the paper's linear-mixing model (genes x iterations / s, %HBM peak)",
        "value": V * args.steps / sec,
        "unit": "genes*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"linear-mixing EM (Section 4.2), V={V} genes, N={N}, K={K_true}, rho=100, seed {seed}",
                   "V": V, "N": N},
        "loglik_last": float(ll[-1]),
        "roofline": {
            "kernel": LM_KERNEL,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("em", LM_SRC),
            "avg_ms": pass_ms,
            "bytes_per_launch": bytes_per_pass,
        },
        "table1": table1,
        "table1_mean_error": sum(t["error"] for t in table1) / len(table1),
        "time_to_convergence_V8000": {"rel_tol": 1e-7, "seconds": conv_s, "iterations": n_conv, "converged": conv,
                                      "loglik": ll_conv},
    }
    if not args.no_cpu:
        from oracle import lmem_oracle as le

        Vs = 1_000_000
        p = le.start(N)
        iters = 0
        t0 = time.perf_counter()
        while True:
            le.loglik(r[:Vs], d[:Vs], p)
            p = le.iterate(r[:Vs], d[:Vs], p)
            iters += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": Vs * iters / el, "unit": "genes*iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iteration(s) with the log-likelihood on the first {Vs} genes of the same data from "
                      f"the start ({el:.1f} s, numpy FP64, one thread)"}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


def gibbs_roofline(V: int, pass_ms: float, bytes_per_pass: float) -> dict:
    """The per-gene Gibbs pass issues far more FP64 instructions per gene (the Philox, Box-Muller and
    factor arithmetic) than its 8 (N + 1) bytes of HBM traffic can hide: it is bound by FP64 issue.
    Achieved: the FP64 instructions of its loop body per gene (counted in the gfx950 assembly of the
    kernel source, recorded with that source's hash) x V per pass time, in lane operations per
    second; peak: 256 CUs x 64 FP64 lanes x 2.4 GHz (the published 78.6 TFLOP/s counts an FMA as
    two)."""
    peak = 256 * 64 * 2.4e9 / 1e12
    try:
        with open(TRAFFIC_FILE) as f:
            isa = json.load(f).get("gibbs_isa")
    except (OSError, ValueError):
        isa = None
    per_gene = isa["fp64_per_gene"] if isa and isa.get("kernel_sha") == kernel_sha(GIBBS_SRC) else None
    achieved = per_gene * V / (pass_ms * 1e-3) / 1e12 if per_gene else None
    hbm = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    return {
        "kernel": GIBBS_KERNEL,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFP64-lane-op/s",
        "frac": achieved / peak if achieved else None,
        "traffic": measured_traffic("gibbs", GIBBS_SRC),
        "avg_ms": pass_ms,
        "fp64_ops_per_gene": per_gene,
        "hbm_achieved_GBs": hbm,
        "hbm_frac": hbm / HBM_PEAK_GBS,
        "bytes_per_launch": bytes_per_pass,
    }


def gibbs_bench(args) -> int:
    """The paper's Gibbs sampler for its linear-mixing model (Section 4.1, eqs 32-40) on the same
    genes as the variational workload: V genes with N = 3 networks, K = (0.1, 0.3), rho = 100.  A
    step is one iteration (every beta_i drawn from its full conditional, then rho, Lambda and K)."""
    import numpy as np
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.gibbs import LinMixGibbs

    V, N, K_true, seed = 10_000_000, 3, (0.1, 0.3), 2
    r, d = synth.linmix_dataset(seed, V, K_true)
    rd, dd = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    h = LinMixGibbs(rd, dd, seed=seed)
    if args.warmup:
        h.iterate(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.iterate(args.steps)
    sec = time.perf_counter() - t0
    pass_ms = h.profile_pass(20)
    h.close()
    bytes_per_pass = 8.0 * V * (N + 1)  # r and d read once, FP64
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    # the Gibbs column of Table 1: its five weight vectors, V = 8000 genes, the paper's 8000
    # iterations (its chain converged in 8000); the posterior mean of K after 1000 discarded
    table1 = []
    TABLE1_GIBBS = [((0.1, 0.3), (0.1011, 0.3003)), ((0.13, 0.25), (0.1234, 0.2311)),
                    ((0.39, 0.54), (0.3829, 0.5312)), ((0.25, 0.16), (0.2441, 0.1948)),
                    ((0.18, 0.29), (0.1822, 0.2643))]
    chain_s = 0.0
    for row, (k_true, k_paper) in enumerate(TABLE1_GIBBS):
        rs, ds = synth.linmix_dataset(1 + row, 8000, k_true)
        hs = LinMixGibbs(torch.from_numpy(rs).cuda(), torch.from_numpy(ds).cuda(), seed=100 + row)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hs.iterate(8000)
        chain_s += time.perf_counter() - t1
        _, Kc, _ = hs.chain(1000, 7000)
        hs.close()
        ke = Kc.mean(0)
        table1.append({"actual": list(k_true), "gibbs": [round(float(v), 4) for v in ke],
                       "error": float(np.linalg.norm(ke - np.array(k_true))), "paper_gibbs": list(k_paper)})
    if args.copy_ref:
        src = torch.ones(96_000_000, dtype=torch.float32, device=rd.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": "Gibbs iterations/s of the paper's linear-mixing model (genes x iterations / s, %HBM peak)",
        "value": V * args.steps / sec,
        "unit": "genes*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"linear-mixing Gibbs (Section 4.1), V={V} genes, N={N}, K={K_true}, rho=100, seed {seed}",
                   "V": V, "N": N},
        "roofline": gibbs_roofline(V, pass_ms, bytes_per_pass),
        "table1": table1,
        "table1_mean_error": sum(t["error"] for t in table1) / len(table1),
        "table1_chain_seconds_per_8000_iterations_V8000": chain_s / len(table1),
    }
    if not args.no_cpu:
        from oracle import gibbs_oracle as go
        from oracle import lmvb_oracle as lo

        Vs = 1_000_000
        pr = lo.default_prior(N)
        c = go.start(N, pr)
        rng = go.Rng(seed)
        iters = 0
        t0 = time.perf_counter()
        while True:
            go.iterate(r[:Vs], d[:Vs], c, pr, rng)
            iters += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": Vs * iters / el, "unit": "genes*iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iteration(s) on the first {Vs} genes of the same data from the start ({el:.1f} s, "
                      f"numpy FP64, one thread)"}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


def figs_bench(args) -> int:
    """The paper's run-time experiment (Section 4, Figs 5-7): its linear-mixing model with N = 3 at
    V = 4000, 5000, 6000, 7000 and 8000 genes, 4000 iterations of VB and of EM and 10,000 of the
    Gibbs sampler, each timed from data already on the device to the last iteration's result on the
    host.  The paper's GTX 1050 and i5-8300H times are printed beside them as context (another
    machine): they are not a target.  At these sizes every kernel lasts a few microseconds, so the
    runs are bound by the fixed costs of the kernels, not by HBM or the ALUs."""
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.gibbs import LinMixGibbs
    from paper_2401_10068_amd.lmem import LinMixEM
    from paper_2401_10068_amd.lmvb import LinMixVB

    paper = {  # seconds: (VB GPU, VB CPU, EM GPU, EM CPU, Gibbs GPU, Gibbs CPU), Figs 5-7
        4000: (62, 424, 53, 330, 201, 1202), 5000: (74, 522, 65, 405, 246, 1490),
        6000: (88, 621, 78, 486, 297, 1785), 7000: (101, 723, 90, 560, 341, 2104),
        8000: (116, 846, 104, 637, 389, 2391)}
    runs = []
    for V in sorted(paper):
        r, d = synth.linmix_dataset(1, V, (0.1, 0.3))
        rd, dd = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = LinMixVB(rd, dd)
        h.init()
        h.sweep(4000)
        h.globals()
        vb = time.perf_counter() - t0
        h.close()
        t0 = time.perf_counter()
        h = LinMixEM(rd, dd)
        h.iterate(4000)
        h.params()
        em = time.perf_counter() - t0
        h.close()
        t0 = time.perf_counter()
        h = LinMixGibbs(rd, dd, seed=1)
        h.iterate(10000)
        h.state()
        gb = time.perf_counter() - t0
        h.close()
        pv = paper[V]
        runs.append({"V": V, "vb_s": vb, "em_s": em, "gibbs_s": gb,
                     "paper_gtx1050_s": {"vb": pv[0], "em": pv[2], "gibbs": pv[4]},
                     "paper_i5_8300h_s": {"vb": pv[1], "em": pv[3], "gibbs": pv[5]}})
    last = runs[-1]
    out = {
        "metric": "seconds for the paper's fixed-iteration runs (Figs 5-7): 4000 VB sweeps at V = 8000",
        "value": last["vb_s"],
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "linear-mixing model, N=3, K=(0.1, 0.3), rho=100, V=4000..8000 genes; VB and EM "
                               "4000 iterations, Gibbs 10000"},
        "runs": runs,
        "roofline": None,
        "note": "bound by the fixed costs of three kernels of a few microseconds per iteration",
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import gibbs_oracle as go
        from oracle import lmem_oracle as le
        from oracle import lmvb_oracle as lo

        r, d = synth.linmix_dataset(1, 8000, (0.1, 0.3))
        pr = lo.default_prior(3)
        n = 200
        t0 = time.perf_counter()
        lo.run(r, d, pr, n)
        vb = (time.perf_counter() - t0) * 4000 / n
        t0 = time.perf_counter()
        le.run(r, d, n)
        em = (time.perf_counter() - t0) * 4000 / n
        t0 = time.perf_counter()
        go.run(r, d, n, seed=1)
        gb = (time.perf_counter() - t0) * 10000 / n
        out["cpu_baseline"] = {
            "value": vb, "unit": "s", "cores": 1, "kind": "oracle",
            "em_s": em, "gibbs_s": gb,
            "sample": f"{n} iterations of each oracle (VB with its bound, EM with its log-likelihood, Gibbs) at "
                      f"V = 8000, scaled to 4000 / 4000 / 10000 iterations (numpy FP64, one thread)"}

    print(json.dumps(out), flush=True)
    return 0


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
    sched = bt.schedule()
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
                    "effective_GBps": bytes_read / t_run / 1e9, "estep_schedule": sched},
        "plain_one_at_a_time": {"sample": int(idx.size), "sample_s": t_plain,
                                "extrapolated_s": t_plain / frac, "sweeps_median": float(np.median(plain_sw)),
                                "max_rel_elbo_diff_vs_batched": max_rel},
        "speedup_batched_vs_plain": (t_plain / frac) / (t_init + t_run),
    }
    print(json.dumps(out), flush=True)
    return 0


def warm_bench(args) -> int:
    """Time to ELBO convergence (1e-6 relative) of 4,096 fresh K=8 datasets: plain GPU CAVI one
    dataset at a time (sample), batched from the standard initialisation, and batched from a
    learned warm start, three side by side: MLPs on per-dataset summary features (per gene:
    moments and 16 nearest-rank quantiles, the workload's definition; moments and 16 rank-bin
    means), and the learned refinement of the standard initialisation (RefineStart).  Plain CAVI is the
    judge: a warm-started dataset is accepted when its bound is within 1e-6 of the plain one (or
    better); the others fall back to plain CAVI, and the warm start's time to matching bounds is
    the warm batch (features + MLP + state + run) plus a batched plain run of the rejected
    datasets.  Each MLP is trained first on generated datasets (reported), or loaded."""
    import numpy as np
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.cavi import Cavi, CaviBatch
    from paper_2401_10068_amd.warmstart import RefineStart, WarmStart

    Ns, Ks, rec, seed = synth.batch_workload("c5eval")
    G, K = rec.G, int(Ks[0])
    kinds = ["quantiles", "bins", "refine", "refine@0.5"] if args.features == "all" else args.features.split(",")
    nets, trained = {}, {}
    for kind in kinds:
        base, step = (kind.split("@")[0], float(kind.split("@")[1])) if "@" in kind else (kind, 1.0)
        if base in trained:  # refine@s: the network trained for refine, another step along its move
            nets[kind] = (trained[base][0], trained[base][1], step)
            continue
        if base == "refine":
            ws = RefineStart(G=G, K=K, max_batch=1024, seed=args.mlp_seed)
            n_train = args.refine_datasets
        else:
            ws = WarmStart(G=G, K=K, max_batch=1024, seed=args.mlp_seed, features=base)
            n_train = args.train_datasets
        train = None
        if args.mlp_params:
            ws.load(args.mlp_params.replace("{kind}", base))
        else:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = ws.train(n_train, batch=1024, lr=args.lr,
                              log_every=max(1, n_train // 1024 // 10),
                              log=lambda m, kind=kind: print(f"[{kind}] {m}", file=sys.stderr, flush=True))
            torch.cuda.synchronize()
            train = {"datasets": n_train, "steps": int(losses.size), "batch": 1024,
                     "seconds": time.perf_counter() - t0, "loss_first": float(losses[0]),
                     "loss_last_avg10": float(losses[-10:].mean())}
            if args.save_mlp:
                ws.save(args.save_mlp.replace("{kind}", base))
        trained[base] = (ws, train)
        nets[kind] = (ws, train, step)
    x, row_off, _, _, _, _, _ = synth.make_batch_gpu(seed, Ns, Ks, rec)
    off_d = row_off.to(x.device)
    torch.cuda.synchronize()

    def batched(ws, xb, Nb, Kb, offb, seed_b, step=1.0):
        bt = CaviBatch(xb, Nb, Kb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if ws is None:
            bt.init_standard(seed_b)
        elif isinstance(ws, RefineStart):
            ws.warm_start(bt, seed_b, step=step)  # the same standard initialisation, then the learned move
        else:
            ws.warm_start(bt, xb, offb)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        sw, el, nconv = bt.run(args.max_sweeps, 1e-6)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        bt.close()
        return {"init_s": t_init, "total_s": t_all, "converged": nconv, "sweeps_total": int(sw.sum()),
                "sweeps_median": float(np.median(sw)), "sweeps_p90": float(np.percentile(sw, 90)),
                "sweeps_max": int(sw.max())}, sw, el

    plain_b, psw, pel = batched(None, x, Ns, Ks, off_d, seed)
    tol = 1e-6 * np.abs(pel)
    results = {}
    for kind, (ws, train, step) in nets.items():
        warm_b, wsw, wel = batched(ws, x, Ns, Ks, off_d, seed, step)
        accepted = wel >= pel - tol
        better = wel > pel + tol
        rej = np.flatnonzero(~accepted)
        fb = {"datasets": int(rej.size), "total_s": 0.0}
        if rej.size:
            # the rejected datasets' rows gathered into a batch of their own, plain from the standard
            # initialisation (the fallback's cost; their plain bounds are those of the plain run)
            parts = [x[int(row_off[b]):int(row_off[b + 1])] for b in rej]
            xr = torch.cat(parts, 0).contiguous()
            offr = torch.from_numpy(np.concatenate([[0], np.cumsum(Ns[rej])]).astype(np.int64)).to(x.device)
            fb_b, _, _ = batched(None, xr, Ns[rej], Ks[rej], offr, seed)
            fb.update(fb_b)
            del xr, parts
        results[kind] = {
            "training": train, "batched_warm": warm_b, "fallback_plain": fb,
            "warm_plus_fallback_s": warm_b["total_s"] + fb["total_s"],
            "acceptance": {"accepted": int(accepted.sum()), "rate": float(accepted.mean()),
                           "strictly_better": int(better.sum()), "datasets": int(Ns.size),
                           "median_rel_elbo_gap": float(np.median((wel - pel) / np.abs(pel)))},
            "sweeps_accepted_warm_vs_plain": [int(wsw[accepted].sum()), int(psw[accepted].sum())],
            "speedup_vs_batched_plain": plain_b["total_s"] / (warm_b["total_s"] + fb["total_s"]),
        }
    idx = np.arange(0, Ns.size, max(1, Ns.size // args.plain_sample))
    t_plain = 0.0
    for b in idx:
        xb = x[int(row_off[b]):int(row_off[b + 1])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cx = Cavi(xb, K)
        cx.init_standard(seed + int(b))
        cx.run(args.max_sweeps, 1e-6)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        cx.close()
    frac = float(Ns[idx].sum() / Ns.sum())
    best = max(results, key=lambda k: results[k]["speedup_vs_batched_plain"])
    nkg = float((psw.astype(np.float64) * Ns * K * G).sum())
    out = {
        "metric": METRIC,
        # the matching bounds are the plain ones: N K G work of the plain sweeps over the best
        # warm start's time to reach them (warm batch + fallback)
        "value": nkg / results[best]["warm_plus_fallback_s"],
        "unit": "N*K*G elems/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "f32 (MLP: bf16 products, f32 accumulate)",
        "config": {"workload": f"{Ns.size} fresh datasets (c5eval): N log-uniform in [{Ns.min()}, {Ns.max()}], "
                               f"K={K}, G={G}, seed {seed}, run to 1e-6"},
        "plain_one_at_a_time": {"sample": int(idx.size), "sample_s": t_plain, "extrapolated_s": t_plain / frac},
        "batched_plain": plain_b,
        "warm": results,
        "best_features": best,
        "speedup_batched_plain_vs_one_at_a_time": (t_plain / frac) / plain_b["total_s"],
    }
    for ws, _ in trained.values():
        ws.close()
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the device reaches its steady clocks only after some tens of milliseconds of sustained work:
    # at c2, the first 100 sweeps after a 10-sweep warm-up averaged 97.7-99.4 us against 92.5 us
    # for every later call, and 93.0 us after a 200-sweep warm-up (about 20 ms)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c2", choices=["small", "c2", "c3", "c4", "c5", "lm", "em", "gibbs", "figs"])
    ap.add_argument("--schedule", type=int, default=None, choices=[0, 1, 2],
                    help="single-dataset workloads: force an E-step schedule (default: the autotuner's choice; "
                         "2 = the screen as a BF16 matrix product, K in 9..16)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--copy-ref", action="store_true",
                    help="after the bench, run an elementwise kernel 3 times that reads and writes "
                         "384,000,000 bytes (reference of known traffic for the hardware byte counters)")
    ap.add_argument("--max-sweeps", type=int, default=10000, help="batched workloads: sweep cap")
    ap.add_argument("--plain-sample", type=int, default=256, help="batched workloads: datasets timed one at a time")
    ap.add_argument("--train-datasets", type=int, default=1_000_000, help="c5: generated datasets to train on")
    ap.add_argument("--lr", type=float, default=1e-3, help="c5: peak learning rate")
    ap.add_argument("--mlp-seed", type=int, default=0, help="c5: MLP initialisation seed")
    ap.add_argument("--mlp-params", default=None,
                    help="c5: load trained MLP parameters (.npy; '{kind}' in the path is replaced by the feature set)")
    ap.add_argument("--save-mlp", default=None, help="c5: save the trained parameters (.npy; '{kind}' as above)")
    ap.add_argument("--features", default="all",
                    help="c5: warm starts to train and compare: 'all' or a comma list of quantiles, bins, refine "
                         "(refine@s: the learned move scaled by s)")
    ap.add_argument("--refine-datasets", type=int, default=300_000,
                    help="c5: generated datasets (run to convergence) the refinement is trained on")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs on one GPU; the sweep "
              "would shard over rows with one all-gather of the statistics per sweep.", file=sys.stderr)
        return 2
    sys.path.insert(0, ROOT)
    if args.workload == "c4":
        return batch_bench(args)
    if args.workload == "c5":
        return warm_bench(args)
    if args.workload == "lm":
        return lm_bench(args)
    if args.workload == "em":
        return em_bench(args)
    if args.workload == "gibbs":
        return gibbs_bench(args)
    if args.workload == "figs":
        return figs_bench(args)
    import torch

    from paper_2401_10068_amd import synth
    from paper_2401_10068_amd.cavi import Cavi

    N, rec, seed = synth.workload(args.workload)
    K, G = rec.K, rec.G
    x, _, _, _, _ = synth.make_dataset_gpu(seed, 0, N, rec)
    torch.cuda.synchronize()
    cx = Cavi(x, K)
    if args.schedule is not None:
        cx.set_schedule(args.schedule)
    cx.init_standard(seed)
    if args.warmup:
        cx.sweep(args.warmup, want_elbo=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    elbo = cx.sweep(args.steps, want_elbo=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0

    est_ms = cx.profile_estep(20)
    sched, sched_ms = cx.schedule()
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
            "schedule": sched,
            "schedule_ms": sched_ms,
        },
    }
    cx.close()
    if args.copy_ref:
        src = torch.ones(96_000_000, dtype=torch.float32, device=x.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    # what a plain copy and a plain read reach on this GPU, beside the E-step's rate
    ref = copy_reference(x.device)
    ref["estep_frac_of_read"] = achieved / ref["read_GBps"]
    out["hbm_reference"] = ref
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
