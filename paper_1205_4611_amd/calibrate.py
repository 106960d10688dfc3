#!/usr/bin/env python3
"""Calibration of the tree depth (the N_d of eq. (Nlevels), Sec. 5.1) on the
device this runs on.

The paper chooses the number of levels from the desired number of sources per
leaf N_d and shows that the best N_d depends on the hardware and grows with the
expansion order p (Sec. 5.1 "Calibration", Sec. 5.2 "Shift operators"):
deeper trees move work from P2P to the shift operators, whose cost grows with
p.  This script times the evaluation of Phi' at the sources over the levels
L-1, L, L+1 around the level rule at N_d = 45, for each order p and order
policy given, and prints one JSON object: per (N, p, policy) the time of every
level, the fastest level and the N_d interval that eq. (Nlevels) maps to it.

  python -m paper_1205_4611_amd.calibrate --sizes 1048576,4194304,16777216 \\
      --orders 17,20,34 --policies fixed,learned

Inputs are the benchmark's 20-cluster distribution (seeded); only the
library's own kernels are timed.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def nd_interval(n: int, L: int):
    """The N_d values for which eq. (Nlevels) gives L levels at n sources:
    8 N_d 4^L >= 5 n > 8 N_d 4^(L-1) (for L >= 1)."""
    lo = -(-5 * n // (8 * 4 ** L))               # smallest N_d with 8 N_d 4^L >= 5 n
    hi = (5 * n - 1) // (8 * 4 ** (L - 1)) if L >= 1 else None  # largest with 8 N_d 4^(L-1) < 5 n
    return lo, hi


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1048576,4194304,16777216")
    ap.add_argument("--orders", default="17,20,34")
    ap.add_argument("--policies", default="fixed,learned")
    ap.add_argument("--steps", type=int, default=5)
    args = ap.parse_args(argv)

    import torch
    from paper_1205_4611_amd import fmm2d, workloads

    f = fmm2d.FMM2D(0)
    model, delta, _ = fmm2d.load_porder_model()
    f.set_porder_model(model, delta)
    w = workloads.WORKLOADS["clusters4M"]
    out = {"device": torch.cuda.get_device_name(0), "workload": "20 Gaussian clusters, Phi' at the sources, "
           "theta 1/2, FP64, swapped leaf criterion", "runs": []}
    for n in (int(x) for x in args.sizes.split(",")):
        src = torch.from_numpy(workloads.points(w["dist"], n, w["seed"])).cuda()
        m = torch.from_numpy(workloads.strengths(n, w["mseed"])).cuda()
        L0 = fmm2d.nlevels(n, 45)
        for p in (int(x) for x in args.orders.split(",")):
            for pol in args.policies.split(","):
                if pol == "learned" and p < fmm2d.PORDER_FEAT_K:
                    continue  # the model needs the coefficients up to k = 20
                times = {}
                for L in (L0 - 1, L0, L0 + 1):
                    if L < 1 or 4 ** L > n:
                        continue
                    opts = fmm2d.make_opts(p=p, levels=L, kernel="harmonic", porder=pol, swap=True)
                    f.eval(src, m, opts=opts, check=True)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(args.steps):
                        f.eval(src, m, opts=opts, check=False)
                    torch.cuda.synchronize()
                    times[L] = (time.perf_counter() - t0) * 1e3 / args.steps
                    f.sync()
                    print("n=%d p=%d %s L=%d: %.3f ms" % (n, p, pol, L, times[L]), file=sys.stderr, flush=True)
                best = min(times, key=times.get)
                lo, hi = nd_interval(n, best)
                out["runs"].append({"n": n, "p": p, "porder": pol, "ms_by_level": times, "best_level": best,
                                    "rule_level_nd45": L0, "nd_interval_for_best": [lo, hi]})
    print(json.dumps(out))
    f.close()


if __name__ == "__main__":
    main()
