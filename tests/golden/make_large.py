#!/usr/bin/env python3
"""Writes the stored expected values of the full-size parity tests
(tests/test_gpu_fullsize.py).  It calls only the CPU oracle (oracle/) and the
seeded input generators (paper_1205_4611_amd/workloads.py); nothing here comes
from the HIP path.

For each measured workload it stores, at 10,000 seeded sample targets:
  dphi   the compensated FP64 direct sum of Phi' (eq. poteval / paireval,
         Sec. 1), the reference of the pointwise TOL metric of Sec. 5.1;
  phi    for the separate-target sets (LOG kernel): the principal direct sum
         of Phi and the branch-consistent direct sum on the oracle tree (the
         branch the far field follows, see the oracle's direct_branch).
For the 16M spiral it also stores SHA-256 digests of every array of the oracle
tree and lists (L = 9, theta = 1/2, swapped leaf criterion), because the
oracle takes about a minute to build that tree: the GPU test hashes its own
topology the same way (topology_digests below) and compares.

Run from the repository root:  python tests/golden/make_large.py [names...]
(about 15 minutes on 8 cores).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NSAMPLE = 10_000
THETA = 0.5


def topology_digests(perm, tperm, sstart, tstart, centre, radius, weak, strong, m2p, p2l):
    """SHA-256 of each topology array in a fixed byte form: indices and
    starts as little-endian int64, geometry as the raw FP64 bits; weak and
    strong are per-level (offsets from 0, indices) pairs, m2p and p2l one
    such pair.  Shared by this script (on the oracle's arrays) and the GPU
    test (on the library's)."""
    def h(*arrays):
        g = hashlib.sha256()
        for a in arrays:
            a = np.asarray(a)
            if a.dtype.kind in "iu":
                a = a.astype("<i8")
            else:
                a = a.astype("<f8") if a.dtype.kind == "f" else a.astype("<c16")
            g.update(np.ascontiguousarray(a).tobytes())
        return g.hexdigest()
    out = {"perm": h(perm), "tperm": h(tperm), "sstart": h(sstart), "tstart": h(tstart),
           "centre": h(centre), "radius": h(radius), "m2p": h(*m2p), "p2l": h(*p2l)}
    for l, (off, idx) in enumerate(weak):
        out["weak%d" % l] = h(off, idx)
    for l, (off, idx) in enumerate(strong):
        out["strong%d" % l] = h(off, idx)
    return out


def make(name):
    import oracle
    from paper_1205_4611_amd import workloads
    w = workloads.WORKLOADS[name]
    src, m, tgt = workloads.workload(name)
    nt = len(src) if tgt is None else len(tgt)
    sel = workloads.sample_indices(nt, NSAMPLE, w["sel_seed"])
    L = oracle.nlevels(len(src), w["nd"])
    out = {"sel": sel, "levels": np.int64(L)}
    t0 = time.time()
    if tgt is None:
        _, d = oracle.direct(src, m, kernel=oracle.KERNEL_HARMONIC, tsel=sel)
        out["dphi"] = d
    else:
        p, d = oracle.direct(src, m, tgt=tgt, kernel=oracle.KERNEL_LOG, tsel=sel)
        out["dphi"] = d
        out["phi"] = p
        T = oracle.Tree(src, L, theta=THETA, tgt=tgt)
        out["phi_branch"] = T.direct_branch(m, sel)
        del T
    print("%s: direct sums at %d targets, %.0f s" % (name, len(sel), time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "direct_%s.npz" % name), **out)
    if name == "spiral16M":
        t0 = time.time()
        T = oracle.Tree(src, L, theta=THETA, swap=True)
        dg = topology_digests(T.perm, T.tperm[:len(src)], T.sstart, T.tstart, T.centre, T.radius, T.weak,
                              T.strong, T.m2p, T.p2l)
        dg["levels"] = L
        dg["swap"] = True
        dg["n_weak"] = int(T.n_weak())
        with open(os.path.join(HERE, "topology_%s.json" % name), "w") as fh:
            json.dump(dg, fh, indent=1, sort_keys=True)
        print("%s: oracle tree and digests, %.0f s" % (name, time.time() - t0), flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["uniform1M", "gauss10_1M", "circle1M", "clusters4M", "spiral16M"]
    for nm in names:
        make(nm)
