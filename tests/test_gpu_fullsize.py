"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (default two-stream schedule, theta 1/2,
levels by eq. (Nlevels) with N_d = 45, swapped leaf criterion for the
at-source workloads).

  clusters4M  N = 2^22, 20 Gaussian clusters, Phi' at the sources (the
              benchmark workload): tree and lists bit-exact against the oracle
              tree; the FMM at p = 20 against the oracle FMM at equal p and
              lists (normwise 1e-12, and pointwise at the sampled targets); the
              FMM with seeded per-pair orders against the oracle at the same
              orders; fixed p = 20 and learned orders against the oracle's
              direct sum at 10,000 sampled sources (pointwise TOL 1e-6,
              Sec. 5.1).
  spiral16M   N = 2^24, 90% on a spiral: tree and lists bit-exact (SHA-256 of
              every topology array against the digests of the oracle tree) and
              the pointwise TOL at 1e-6 (p = 20, fixed and learned) and 1e-10
              (p = 34) against the oracle's direct sum.
  *1M         N = M = 2^20 with separate evaluation points (uniform, 10
              Gaussians, noisy unit circle), LOG kernel: tree bit-exact against
              the oracle tree, Phi' at TOL 1e-6 (p = 20) and 1e-10 (p = 34)
              pointwise against the direct sum, Phi against the
              branch-consistent direct sum.

The direct sums (and the 16M digests) are stored in tests/golden/ by
tests/golden/make_large.py, which calls only the oracle.
"""
import json
import os

import numpy as np
import pytest

from paper_1205_4611_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dev(z):
    return None if z is None else torch.from_numpy(np.ascontiguousarray(z, dtype=np.complex128)).cuda()


def host(t):
    return None if t is None else t.cpu().numpy()


def nrm(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def ptw(a, b):
    """Pointwise relative error max_i |a_i - b_i| / |b_i| (the TOL metric)."""
    return float(np.max(np.abs(a - b) / np.abs(b)))


def golden(name):
    with np.load(os.path.join(GOLDEN, "direct_%s.npz" % name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_4611_amd import fmm2d
    f = fmm2d.FMM2D(0)
    yield f
    f.close()


def _compare_topology(orc, top, T, L):
    assert np.array_equal(top["perm"], T.perm)
    nt = T.nt or T.ns
    assert np.array_equal(top["tperm"][:nt], T.tperm[:nt])
    assert np.array_equal(top["sstart"].astype(np.int64), T.sstart)
    assert np.array_equal(top["tstart"].astype(np.int64), T.tstart)
    assert np.array_equal(top["centre"].view(np.uint64), T.centre.view(np.uint64))
    assert np.array_equal(top["radius"].view(np.uint64), T.radius.view(np.uint64))
    for l in range(L + 1):
        so = orc.start_offset(l)
        for key, lists in (("weak", T.weak), ("strong", T.strong)):
            off = top[key + "_off"][so:so + 4 ** l + 1].astype(np.int64)
            ro, ri = lists[l]
            assert np.array_equal(off - off[0], ro), (key, l)
            assert np.array_equal(top[key + "_idx"][off[0]:off[-1]], ri), (key, l)
    for key, lst in (("m2p", T.m2p), ("p2l", T.p2l)):
        off = top[key + "_off"].astype(np.int64)
        assert np.array_equal(off, lst[0]), key
        assert np.array_equal(top[key + "_idx"][:off[-1]], lst[1]), key


# ------------------------------------------------------------- clusters4M
@pytest.fixture(scope="module")
def c4m(orc):
    src, m, _ = workloads.workload("clusters4M")
    L = orc.nlevels(len(src), 45)
    print("clusters4M: oracle tree L=%d" % L, flush=True)
    return dict(src=src, m=m, L=L, T=orc.Tree(src, L, swap=True), g=golden("clusters4M"),
                dsrc=dev(src), dm=dev(m))


def test_clusters4M_topology_and_fixed_order(fmm, orc, c4m):
    L, T, g = c4m["L"], c4m["T"], c4m["g"]
    assert L == 8
    _, gd = fmm.eval(c4m["dsrc"], c4m["dm"], p=20, levels=-1, leaf_target=45, kernel="harmonic", swap=True)
    _compare_topology(orc, fmm.topology(), T, L)
    print("clusters4M: topology bit-exact; oracle FMM p=20", flush=True)
    _, rd = T.eval(c4m["m"], 20, orc.KERNEL_HARMONIC)
    d = host(gd)
    sel = g["sel"]
    e_n, e_s = nrm(d, rd), ptw(d[sel], rd[sel])
    e_tol = ptw(d[sel], g["dphi"])
    print("clusters4M p=20: vs oracle FMM normwise %.2e, pointwise at the sample %.2e; vs direct %.2e"
          % (e_n, e_s, e_tol))
    assert e_n < 1e-12
    assert e_s < 1e-10  # rounding order only, at 10,000 targets
    assert e_tol < 1e-6


def test_clusters4M_given_orders(fmm, orc, c4m):
    T = c4m["T"]
    q = workloads.pair_orders(T.n_weak(), 4, 20, 86)
    _, rd = T.eval(c4m["m"], 20, orc.KERNEL_HARMONIC, orders=q)
    fmm.set_pair_orders(torch.from_numpy(q).cuda())
    _, gd = fmm.eval(c4m["dsrc"], c4m["dm"], p=20, levels=-1, leaf_target=45, kernel="harmonic", swap=True,
                     porder="given")
    fmm.set_pair_orders(None)
    e = nrm(host(gd), rd)
    print("clusters4M given orders: normwise %.2e" % e)
    assert e < 1e-12


def test_clusters4M_learned_meets_tol(fmm, c4m):
    from paper_1205_4611_amd import fmm2d
    model, delta, _ = fmm2d.load_porder_model()
    fmm.set_porder_model(model, delta)
    g = c4m["g"]
    _, gd = fmm.eval(c4m["dsrc"], c4m["dm"], p=20, levels=-1, leaf_target=45, kernel="harmonic", swap=True,
                     porder="learned")
    st = fmm.stats()
    fmm.set_porder_model(None)
    assert st["used_model"] == 1
    hist = np.array(st["p_hist"][:21], np.float64)
    e = ptw(host(gd)[g["sel"]], g["dphi"])
    print("clusters4M learned: pointwise %.2e at mean order %.2f" % (e, (hist * np.arange(21)).sum() / hist.sum()))
    assert e < 1e-6


# -------------------------------------------------------------- spiral16M
@pytest.fixture(scope="module")
def s16m():
    src, m, _ = workloads.workload("spiral16M")
    with open(os.path.join(GOLDEN, "topology_spiral16M.json")) as fh:
        dg = json.load(fh)
    return dict(dsrc=dev(src), dm=dev(m), g=golden("spiral16M"), dg=dg)


def _digests(top, L):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_large", os.path.join(GOLDEN, "make_large.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    weak, strong = [], []
    for l in range(L + 1):
        so = (4 ** l - 1) // 3 + l
        for key, out in (("weak", weak), ("strong", strong)):
            off = top[key + "_off"][so:so + 4 ** l + 1].astype(np.int64)
            out.append((off - off[0], top[key + "_idx"][off[0]:off[-1]]))
    lists = []
    for key in ("m2p", "p2l"):
        off = top[key + "_off"].astype(np.int64)
        lists.append((off, top[key + "_idx"][:off[-1]]))
    return mk.topology_digests(top["perm"], top["tperm"], top["sstart"], top["tstart"], top["centre"],
                               top["radius"], weak, strong, lists[0], lists[1])


def test_spiral16M_topology_bitexact(fmm, s16m):
    dg = s16m["dg"]
    _, gd = fmm.eval(s16m["dsrc"], s16m["dm"], p=20, levels=-1, leaf_target=45, kernel="harmonic", swap=True)
    top = fmm.topology()
    assert top["levels"] == dg["levels"] == 9
    mine = _digests(top, 9)
    bad = [k for k in mine if mine[k] != dg[k]]
    assert not bad, bad
    e = ptw(host(gd)[s16m["g"]["sel"]], s16m["g"]["dphi"])
    print("spiral16M p=20: topology bit-exact, pointwise %.2e" % e)
    assert e < 1e-6


@pytest.mark.parametrize("tol,p,porder", [(1e-6, 20, "learned"), (1e-10, 34, "fixed")])
def test_spiral16M_tol(fmm, s16m, tol, p, porder):
    from paper_1205_4611_amd import fmm2d
    if porder == "learned":
        model, delta, _ = fmm2d.load_porder_model()
        fmm.set_porder_model(model, delta)
    _, gd = fmm.eval(s16m["dsrc"], s16m["dm"], p=p, levels=-1, leaf_target=45, kernel="harmonic", swap=True,
                     porder=porder)
    st = fmm.stats()
    fmm.set_porder_model(None)
    if porder == "learned":
        assert st["used_model"] == 1
    e = ptw(host(gd)[s16m["g"]["sel"]], s16m["g"]["dphi"])
    print("spiral16M TOL %.0e (p=%d, %s): pointwise %.2e" % (tol, p, porder, e))
    assert e < tol


# ------------------------------------------------------- 1M, separate targets
@pytest.mark.parametrize("name", ["uniform1M", "gauss10_1M", "circle1M"])
def test_separate_targets_1M(fmm, orc, name):
    src, m, tgt = workloads.workload(name)
    g = golden(name)
    L = orc.nlevels(len(src), 45)
    assert L == 7 and int(g["levels"]) == L
    ds, dm, dt = dev(src), dev(m), dev(tgt)
    sel = g["sel"]
    gp, gd = fmm.eval(ds, dm, dt, p=20, levels=-1, leaf_target=45, kernel="log")
    top = fmm.topology()
    print("%s: oracle tree" % name, flush=True)
    _compare_topology(orc, top, orc.Tree(src, L, tgt=tgt), L)
    res = {}
    for tol, p in ((1e-6, 20), (1e-10, 34)):
        gp, gd = fmm.eval(ds, dm, dt, p=p, levels=-1, leaf_target=45, kernel="log")
        e_d = ptw(host(gd)[sel], g["dphi"])
        e_p = ptw(host(gp)[sel], g["phi_branch"])
        res[tol] = (e_d, e_p)
        print("%s TOL %.0e p=%d: Phi' pointwise %.2e, Phi (branch-consistent) pointwise %.2e"
              % (name, tol, p, e_d, e_p))
    for tol, (e_d, e_p) in res.items():
        assert e_d < tol and e_p < tol, (tol, e_d, e_p)
