#!/usr/bin/env python3
"""Benchmark of the adaptive 2D FMM evaluation on one MI355X.

One step = one full evaluation (tree build, lists, P2M, M2M, M2L, L2L, L2P,
P2P, near+far sum) of Phi' for N = 2^22 sources drawn from 20 Gaussian
clusters, evaluated at the sources, with inputs resident in HBM.  The headline
path is the mixed-precision one (FP32 near field and FP32 M2L contraction);
the plain FP64 path is timed beside it.  Each run's error is measured against
a device FP64 direct sum on 10,000 seeded random targets.

Prints one JSON line (see the keys below).  `python bench.py --gpus N` with
N > 1 exits: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "Mparticles/s, N=4M clustered, rel.err≤1e-6: mixed+learned-p vs plain FP64 FMM"
WORKLOAD = "clusters4M"
PEAK = {"f64": 78.6, "f32": 157.3}  # TFLOP/s, MI355X vector (FP32 figure assumes packed issue)
HBM_PEAK = 8000.0  # GB/s


def p2p_flops_per_pair(kernel: str) -> float:
    """Algorithmic flops of one near-field pair (harmonic): w = y - x (2),
    |w|^2 (3), 1/|w|^2 (1), m conj(w) (6), scale and accumulate (4)."""
    return 16.0 if kernel == "harmonic" else 16.0 + 10.0


def l2p_flops_per_target(kernel: str, p: int) -> float:
    """Horner evaluation of the local expansion: one complex multiply-add per
    order (8 flops), twice with the derivative."""
    return 8.0 * p * (1 if kernel == "harmonic" else 2)


def run_path(f, fmm2d, src, m, kernel, p, precision, porder, steps, warmup):
    import torch
    opts = fmm2d.make_opts(p=p, levels=-1, leaf_target=45, kernel=kernel, precision=precision,
                           porder=porder, timing=True, swap=True)
    out = None
    for _ in range(warmup):
        out = f.eval(src, m, opts=opts, check=True)
    torch.cuda.synchronize()
    phases = {k: 0.0 for k in fmm2d.PHASES}
    t0 = time.perf_counter()
    for _ in range(steps):
        out = f.eval(src, m, opts=opts, check=False)
        st = f.stats()  # synchronises; per-phase device times from HIP events on the eval stream
        for k, v in st["ms"].items():
            phases[k] += v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    phases = {k: v / steps for k, v in phases.items()}
    return out, ms, phases, st


def errors(f, src, m, dphi, sel, kernel):
    """Pointwise and normwise relative error of Phi' against the device FP64
    direct sum at the selected targets."""
    import torch
    _, ref = f.direct(src, m, tsel=sel, kernel="harmonic")
    got = dphi[sel]
    e = (got - ref).abs()
    pt = (e / ref.abs()).max().item()
    nrm = (e.max() / ref.abs().max()).item()
    q = torch.quantile((e / ref.abs()).float(), 0.999).item()
    return {"pt": pt, "nrm": nrm, "pt_q999": q}


def cpu_baseline(n_sample: int, p: int):
    """The oracle (plain C, FP64, OpenMP over all host cores) on a bounded
    sample of the same workload: the same distribution at n_sample points."""
    import oracle
    from paper_1205_4611_amd import workloads
    oracle.build()
    w = workloads.WORKLOADS[WORKLOAD]
    src = workloads.points(w["dist"], n_sample, w["seed"])
    m = workloads.strengths(n_sample, w["mseed"])
    L = oracle.nlevels(n_sample, 45)
    t0 = time.perf_counter()
    T = oracle.Tree(src, L)
    T.eval(m, p, oracle.KERNEL_HARMONIC)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count()
    return {"value": n_sample / dt / 1e6, "unit": "Mparticles/s", "cores": cores, "kind": "oracle",
            "sample": "oracle FMM (tree+lists+eval, p=%d, harmonic) on %d points of the same 20-cluster "
                      "distribution, %.1f s wall" % (p, n_sample, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="override N (default 2^22)")
    ap.add_argument("--p", type=int, default=17)
    ap.add_argument("--kernel", default="harmonic", choices=["harmonic", "log"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU path is not part of this build "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1205_4611_amd import fmm2d, workloads

    w = workloads.WORKLOADS[WORKLOAD]
    n = args.n or w["n"]
    src_h = workloads.points(w["dist"], n, w["seed"])
    m_h = workloads.strengths(n, w["mseed"])
    sel_h = workloads.sample_indices(n, 10_000, w["sel_seed"])
    src = torch.from_numpy(src_h).cuda()
    m = torch.from_numpy(m_h).cuda()
    sel = torch.from_numpy(sel_h).cuda()
    f = fmm2d.FMM2D(0)

    res = {}
    for name, prec, porder in (("fp64", "fp64", "fixed"), ("mixed", "mixed", "fixed")):
        out, ms, ph, st = run_path(f, fmm2d, src, m, args.kernel, args.p, prec, porder, args.steps, args.warmup)
        err = errors(f, src, m, out[1], sel, args.kernel)
        res[name] = dict(ms=ms, phases=ph, stats=st, err=err)

    head = res["mixed"]
    st = head["stats"]
    L = fmm2d.nlevels(n, 45)
    pairs = st["n_p2p_pairs"]
    flops = pairs * p2p_flops_per_pair(args.kernel) + n * l2p_flops_per_target(args.kernel, args.p)
    p2p_ms = head["phases"]["p2p"]
    achieved = flops / (p2p_ms * 1e-3) / 1e12
    fp64 = res["fp64"]
    a64 = flops / (fp64["phases"]["p2p"] * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": n / (head["ms"] * 1e-3) / 1e6,
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: N=%d sources, 20 Gaussian clusters, Phi' at the sources" % (WORKLOAD, n),
                   "kernel": args.kernel, "theta": 0.5, "p": args.p, "levels": L, "leaf_target": 45,
                   "path": "mixed (FP32 P2P + FP32 MFMA M2L), fixed p"},
        "err": head["err"],
        "fp64": {"value": n / (fp64["ms"] * 1e-3) / 1e6, "ms_per_step": fp64["ms"], "err": fp64["err"],
                 "phases_ms": fp64["phases"],
                 "p2p_roofline": {"bound": "alu", "achieved": a64, "peak": PEAK["f64"], "unit": "TFLOP/s",
                                  "frac": a64 / PEAK["f64"]}},
        "speedup_vs_fp64": fp64["ms"] / head["ms"],
        "phases_ms": head["phases"],
        "counts": {"m2l_pairs": st["n_weak"], "p2p_leaf_pairs": st["n_strong"], "m2p_leaf_pairs": st["n_m2p"],
                   "p2l_leaf_pairs": st["n_p2l"], "p2p_pairs": pairs},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK["f32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["f32"], "traffic": None,
                     "kernel": "k_p2p32 (near field + L2P)",
                     "flops_per_launch": flops},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, args.p)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
