"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each pin_* takes the oracle module and raises AssertionError when the oracle
disagrees with a closed form, an exact identity, a worked example or a
brute-force computation written independently here.  test_oracle.py runs them
on the oracle as it is; test_oracle_mutations.py plants plausible mistakes in
copies of the oracle's C source and checks that some pin catches each one.
"""
from __future__ import annotations

import cmath
import math
import os

import numpy as np

from paper_1205_4611_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- level rule
def pin_level_rule(orc):
    """Worked example of eq. (Nlevels), Sec. 5.1 (golden/level_rule.txt)."""
    for line in open(os.path.join(GOLDEN, "level_rule.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, nd, L = (int(x) for x in line.split())
        got = orc.nlevels(n, nd)
        assert got == L, "levels(%d, %d) = %d, paper says %d" % (n, nd, got, L)


# ---------------------------------------------------------------- direct sum
def pin_direct_roots_of_unity(orc):
    """Closed form: n unit sources at the n-th roots of unity.  At a real y > 1,
    sum log(y - w_k) = log(y^n - 1) and sum 1/(y - w_k) = n y^(n-1)/(y^n - 1); at
    y = 0 the derivative sum vanishes."""
    n = 24
    src = np.exp(2j * np.pi * np.arange(n) / n)
    m = np.ones(n, complex)
    tgt = np.array([1.7, 3.0, 0.0 + 0.0j])
    phi, dphi = orc.direct(src, m, tgt=tgt, kernel=orc.KERNEL_LOG)
    for k, y in enumerate(tgt[:2]):
        y = y.real
        assert abs(phi[k] - math.log(y ** n - 1)) < 1e-12 * abs(math.log(y ** n - 1))
        assert abs(dphi[k] - n * y ** (n - 1) / (y ** n - 1)) < 1e-12 * abs(n * y ** (n - 1) / (y ** n - 1))
    assert abs(dphi[2]) < 1e-13


def pin_direct_bruteforce(orc):
    """Plain Python (cmath) double loop on a tiny input, with a target that
    coincides with a source (excluded) and evaluation at the sources."""
    src = workloads.points("uniform", 40, 11)
    m = workloads.strengths(40, 12)
    tgt = np.concatenate([workloads.points("uniform", 7, 13), src[3:4]])
    for at_src in (False, True):
        T = src if at_src else tgt
        phi, dphi = orc.direct(src, m, tgt=None if at_src else tgt, kernel=orc.KERNEL_LOG)
        ref_p = np.zeros(len(T), complex)
        ref_d = np.zeros(len(T), complex)
        for i, y in enumerate(T):
            for x, mj in zip(src, m):
                if x == y:
                    continue
                ref_p[i] += mj * cmath.log(y - x)
                ref_d[i] += mj / (y - x)
        assert _rel(phi, ref_p) < 1e-13 and _rel(dphi, ref_d) < 1e-13
        _, dh = orc.direct(src, m, tgt=None if at_src else tgt, kernel=orc.KERNEL_HARMONIC)
        assert _rel(dh, ref_d) < 1e-13


# ---------------------------------------------------------------- expansions
def _cluster(seed, n=30, c=0.3 + 0.4j, rad=0.05):
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = rng.uniform(0, 2 * np.pi, n)
    r = rad * np.sqrt(rng.uniform(0, 1, n))
    x = c + r * np.exp(1j * ang)
    m = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return x, m


def pin_p2m_far_field(orc):
    """A multipole evaluated far away equals the direct sum within the
    truncated-series bound: with q = rho/|z-c|, the harmonic tail is at most
    sum|m| q^p / (|z-c| (1-q)) and the log tail at most sum|m| q^(p+1)/((p+1)(1-q))."""
    c = 0.3 + 0.4j
    x, m = _cluster(1, c=c)
    rho = float(np.max(np.abs(x - c)))
    am = float(np.sum(np.abs(m)))
    for p in (4, 10, 20):
        for z in (0.9 + 0.1j, -0.5 + 1.2j, 0.3 + 0.6j):
            q = rho / abs(z - c)
            ah = orc.p2m(orc.KERNEL_HARMONIC, p, c, x, m)
            vh, _ = orc.eval_multipole(p, ah, c, z)
            ref_d = np.sum(m / (z - x))
            bound_h = am * q ** p / (abs(z - c) * (1 - q))
            assert abs(vh - ref_d) <= 1.01 * bound_h + 1e-14 * abs(ref_d)
            al = orc.p2m(orc.KERNEL_LOG, p, c, x, m)
            vl, dl = orc.eval_multipole(p, al, c, z)
            ref_p = np.sum(m * np.log(z - x))
            bound_l = am * q ** (p + 1) / ((p + 1) * (1 - q))
            # same branch: z - c and z - x lie in a half plane around z - c
            assert abs(vl - ref_p) <= 1.01 * bound_l + 1e-14 * abs(ref_p)
            # derivative of the LOG multipole is the harmonic field: tail <= sum|m| q^(p+1)/(|z-c|(1-q))
            assert abs(dl - ref_d) <= 1.01 * am * q ** (p + 1) / (abs(z - c) * (1 - q)) + 1e-14 * abs(ref_d)


def pin_m2m_exact(orc):
    """M2M is exact: the multipole of the union about the parent centre equals
    the sum of the shifted children's multipoles (both kernels)."""
    cp = 0.5 + 0.5j
    kids = [(0.4 + 0.45j, 2), (0.62 + 0.41j, 3), (0.55 + 0.6j, 4), (0.43 + 0.58j, 5)]
    for kernel in (orc.KERNEL_LOG, orc.KERNEL_HARMONIC):
        for p in (5, 17, 30):
            tot = np.zeros(p + 1, complex)
            allx, allm = [], []
            for cc, seed in kids:
                x, m = _cluster(seed, n=12, c=cc, rad=0.04)
                allx.append(x)
                allm.append(m)
                a = orc.p2m(kernel, p, cc, x, m)
                tot = orc.m2m(p, a, cc - cp, out=tot)
            ref = orc.p2m(kernel, p, cp, np.concatenate(allx), np.concatenate(allm))
            assert _rel(tot, ref) < 1e-13, (kernel, p, _rel(tot, ref))


def pin_l2l_exact(orc):
    """L2L is exact: a re-centred polynomial takes the same values."""
    rng = np.random.Generator(np.random.PCG64(7))
    for p in (3, 17, 33):
        b = rng.standard_normal(p + 1) + 1j * rng.standard_normal(p + 1)
        b /= 2.0 ** np.arange(p + 1)  # keep terms O(1) on |w| <= 1
        cp, cc = 0.1 - 0.2j, 0.35 - 0.05j
        bc = orc.l2l(p, b, cc - cp)
        for z in (0.3 + 0.1j, 0.5 - 0.3j, 0.2 - 0.2j):
            v0, d0 = orc.eval_local(p, b, cp, z)
            v1, d1 = orc.eval_local(p, bc, cc, z)
            assert abs(v0 - v1) <= 1e-13 * max(1.0, abs(v0))
            assert abs(d0 - d1) <= 1e-13 * max(1.0, abs(d0))


def pin_m2l_closed_forms(orc):
    """Closed-form re-expansions about c_T, rho = c_T - c_S, w = z - c_T:
       log(z - c_S)      = Log rho + sum_{l>=1} (-1)^(l+1) (w/rho)^l / l
       1/(z - c_S)       = sum_l (-1)^l w^l / rho^(l+1)
       1/(z - c_S)^2     = sum_l (-1)^l (l+1) w^l / rho^(l+2)"""
    p = 12
    for rho in (0.7 - 0.4j, -0.9 + 0.2j, -0.3 - 0.8j):
        e0 = np.zeros(p + 1, complex); e0[0] = 1
        e1 = np.zeros(p + 1, complex); e1[1] = 1
        e2 = np.zeros(p + 1, complex); e2[2] = 1
        l = np.arange(p + 1)
        b0 = orc.m2l(p, e0, rho)
        ref0 = np.zeros(p + 1, complex)
        ref0[0] = cmath.log(rho)
        ref0[1:] = (-1.0) ** (l[1:] + 1) / (l[1:] * rho ** l[1:])
        assert _rel(b0, ref0) < 1e-14
        assert _rel(orc.m2l(p, e1, rho), (-1.0) ** l / rho ** (l + 1)) < 1e-14
        assert _rel(orc.m2l(p, e2, rho), (-1.0) ** l * (l + 1) / rho ** (l + 2)) < 1e-14


def pin_m2l_convergence(orc):
    """P2M -> M2L -> L2P of a source cluster against the direct sum at points of
    a well-separated target disc: the error falls geometrically in p and stays
    below the a-priori bound (|x|+|y|)^(p+1)/(1-|x|-|y|) times sum|m|/d."""
    cS, cT = 0.2 + 0.2j, 0.8 + 0.55j
    x, m = _cluster(9, n=40, c=cS, rad=0.08)
    rS = float(np.max(np.abs(x - cS)))
    rT = 0.08
    d = abs(cT - cS)
    ratio = (rS + rT) / d
    zs = cT + rT * np.exp(1j * np.linspace(0, 2 * np.pi, 9)[:-1])
    ref_d = np.array([np.sum(m / (z - x)) for z in zs])
    ref_p = np.array([np.sum(m * np.log(z - x)) for z in zs])
    am = float(np.sum(np.abs(m)))
    errs = []
    for p in (4, 8, 12, 16, 20):
        ah = orc.p2m(orc.KERNEL_HARMONIC, p, cS, x, m)
        bh = orc.m2l(p, ah, cT - cS)
        vh = np.array([orc.eval_local(p, bh, cT, z)[0] for z in zs])
        e = float(np.max(np.abs(vh - ref_d)))
        errs.append(e)
        assert e <= 2.0 * am / d * ratio ** (p + 1) / (1 - ratio) / (1 - ratio), (p, e)
        al = orc.p2m(orc.KERNEL_LOG, p, cS, x, m)
        bl = orc.m2l(p, al, cT - cS)
        vals = [orc.eval_local(p, bl, cT, z) for z in zs]
        vl = np.array([v[0] for v in vals])
        dl = np.array([v[1] for v in vals])
        assert float(np.max(np.abs(vl - ref_p))) <= 2.0 * am * ratio ** (p + 1) / (1 - ratio) ** 2
        assert float(np.max(np.abs(dl - ref_d))) <= 4.0 * am / d * (p + 2) * ratio ** (p + 1) / (1 - ratio) ** 2
    # geometric decay: fitted ratio per order below the bound ratio
    slope = np.polyfit(np.arange(5) * 4.0, np.log(np.maximum(errs, 1e-300)), 1)[0]
    assert math.exp(slope) <= ratio * 1.05, (math.exp(slope), ratio)


# ---------------------------------------------------------------- tree
def _read_hand():
    pts = {}
    rows = {}
    for line in open(os.path.join(GOLDEN, "tree_hand.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        if key == "pt":
            pts[int(vals[0])] = float(vals[1]) + 1j * float(vals[2])
        else:
            rows.setdefault(key, []).append(vals)
    src = np.array([pts[i] for i in range(len(pts))])
    return src, rows


def pin_tree_hand(orc):
    """Hand-worked 8-point tree and lists (golden/tree_hand.txt)."""
    src, rows = _read_hand()
    T = orc.Tree(src, 1)
    assert list(T.perm) == [int(v) for v in rows["perm"][0]]
    assert list(T.starts(1)) == [int(v) for v in rows["start1"][0]]
    c = np.array([float(v) for v in rows["centre1"][0]])
    got = T.centre[T.boxes(1)]
    assert np.allclose(got.real, c[0::2], rtol=0, atol=1e-15) and np.allclose(got.imag, c[1::2], rtol=0, atol=1e-15)
    r2 = np.array([float(v) for v in rows["radius_sq1"][0]])
    assert np.allclose(T.radius[T.boxes(1)] ** 2, r2, rtol=1e-14, atol=0)
    off, idx = T.weak[1]
    for vals in rows["weak1"]:
        b = int(vals[0].rstrip(":"))
        assert list(idx[off[b]:off[b + 1]]) == [int(v) for v in vals[1:]]
    soff, sidx = T.strong[1]
    for b in range(4):
        assert list(sidx[soff[b]:soff[b + 1]]) == [b]


def _check_tree(orc, src, tgt, L):
    T = orc.Tree(src, L, tgt=tgt)
    ns = len(src)
    assert sorted(T.perm.tolist()) == list(range(ns))
    tg = src if tgt is None else tgt
    if tgt is not None:
        assert sorted(T.tperm.tolist()) == list(range(len(tgt)))
    for l in range(L + 1):
        st = T.starts(l)
        tst = T.starts(l, targets=True)
        assert st[0] == 0 and st[-1] == ns
        if l < L:
            ch = T.starts(l + 1)
            # children partition their parent, counts from two exact halvings
            for b in range(4 ** l):
                n = st[b + 1] - st[b]
                c = np.diff(ch[4 * b:4 * b + 5])
                lo, hi = n // 2, n - n // 2
                assert list(c) == [lo // 2, lo - lo // 2, hi // 2, hi - hi // 2]
                tc = tst[b + 1] - tst[b]
                assert T.starts(l + 1, targets=True)[4 * b + 4] - T.starts(l + 1, targets=True)[4 * b] == tc
        cen = T.centre[T.boxes(l)]
        rad = T.radius[T.boxes(l)]
        for b in range(4 ** l):
            idx = T.perm[st[b]:st[b + 1]]
            if l == L:
                assert np.all(np.diff(idx) > 0), "inside a leaf, sources are in index order"
            pts = src[idx]
            if tgt is not None:
                pts = np.concatenate([pts, tg[T.tperm[tst[b]:tst[b + 1]]]])
            x0, x1, y0, y1 = pts.real.min(), pts.real.max(), pts.imag.min(), pts.imag.max()
            # tight rectangle: the box is the rectangle's midpoint / half diagonal
            assert abs(cen[b] - complex(0.5 * (x0 + x1), 0.5 * (y0 + y1))) <= 4e-16
            assert abs(rad[b] - 0.5 * math.hypot(x1 - x0, y1 - y0)) <= 4e-16 * max(1, rad[b])
            assert np.all(np.abs(pts - cen[b]) <= rad[b] * (1 + 1e-12) + 1e-300)
    return T


def _check_split_rule(orc, src, L):
    """The two splits of each box are exact (coordinate, index) rank splits
    along the longer side of the set's tight rectangle."""
    T = orc.Tree(src, L)
    for l in range(L):
        st = T.starts(l)
        ch = T.starts(l + 1)
        for b in range(4 ** l):
            par = T.perm[st[b]:st[b + 1]]
            lo = T.perm[ch[4 * b]:ch[4 * b + 2]]
            hi = T.perm[ch[4 * b + 2]:ch[4 * b + 4]]
            for s_set, lo_set, hi_set in ((par, lo, hi),
                                          (lo, T.perm[ch[4 * b]:ch[4 * b + 1]], T.perm[ch[4 * b + 1]:ch[4 * b + 2]]),
                                          (hi, T.perm[ch[4 * b + 2]:ch[4 * b + 3]], T.perm[ch[4 * b + 3]:ch[4 * b + 4]])):
                p = src[s_set]
                ax = 0 if (p.real.max() - p.real.min()) >= (p.imag.max() - p.imag.min()) else 1
                key = (lambda i: (src[i].real, i)) if ax == 0 else (lambda i: (src[i].imag, i))
                order = sorted(s_set.tolist(), key=key)
                k = len(order) // 2
                assert sorted(lo_set.tolist()) == sorted(order[:k])
                assert sorted(hi_set.tolist()) == sorted(order[k:])


def pin_tree_invariants(orc):
    for dist, n, L in (("uniform", 700, 2), ("clusters", 1000, 3), ("spiral", 517, 2)):
        src = workloads.points(dist, n, 21)
        _check_tree(orc, src, None, L)
        _check_split_rule(orc, src, L)
    src = workloads.points("gauss10", 600, 22)
    tgt = workloads.points("gauss10", 450, 23)
    _check_tree(orc, src, tgt, 2)


def pin_tree_targets_on_pivot(orc):
    """Separate targets follow the split coordinate: a target exactly at the
    first hi source's coordinate goes to hi.  4 sources on a line, L = 1."""
    src = np.array([0.0 + 0.0j, 1.0 + 0.0j, 2.0 + 0.1j, 3.0 + 0.0j])
    tgt = np.array([2.0 + 0.05j, 1.0 + 0.02j, 0.5 + 0.0j])
    T = orc.Tree(src, 1, tgt=tgt)
    # root split on x: lo = {0,1}, hi = {2,3}, pivot x = 2: target 0 -> hi, targets 1, 2 -> lo
    tst = T.starts(1, targets=True)
    lo_t = set(T.tperm[tst[0]:tst[2]].tolist())
    hi_t = set(T.tperm[tst[2]:tst[4]].tolist())
    assert lo_t == {1, 2} and hi_t == {0}, (lo_t, hi_t)


# ---------------------------------------------------------------- lists
def _theta_ok(cb, rb, cs, rs, theta):
    d = abs(cb - cs)
    return d > 0 and max(rb, rs) + theta * min(rb, rs) <= theta * d


def pin_lists(orc):
    """Interaction lists: directed lists are symmetric, each weak pair passes
    the theta-criterion, each strong pair fails it or is the box itself, the
    parents of every pair are strong, and every (target leaf, source leaf) pair
    is handled exactly once (one M2L at one level, or P2P)."""
    for dist, n, L, tgt in (("uniform", 2000, 3, None), ("clusters", 3000, 4, None),
                            ("gauss10", 1500, 3, ("gauss10", 31))):
        src = workloads.points(dist, n, 30)
        tg = None if tgt is None else workloads.points(tgt[0], 1200, tgt[1])
        T = orc.Tree(src, L, tgt=tg)
        cov = np.zeros((4 ** L, 4 ** L), np.int64)
        for l in range(1, L + 1):
            woff, widx = T.weak[l]
            soff, sidx = T.strong[l]
            cen = T.centre[T.boxes(l)]
            rad = T.radius[T.boxes(l)]
            W = set()
            S = set()
            psoff, psidx = T.strong[l - 1]
            for b in range(4 ** l):
                wl = widx[woff[b]:woff[b + 1]]
                sl = sidx[soff[b]:soff[b + 1]]
                assert np.all(np.diff(wl) > 0) and np.all(np.diff(sl) > 0)
                assert b in sl
                parent_strong = set(psidx[psoff[b // 4]:psoff[b // 4 + 1]].tolist())
                for s in wl:
                    assert _theta_ok(cen[b], rad[b], cen[s], rad[s], 0.5)
                    assert s // 4 in parent_strong
                    W.add((b, int(s)))
                for s in sl:
                    assert s == b or not _theta_ok(cen[b], rad[b], cen[s], rad[s], 0.5)
                    assert s // 4 in parent_strong
                    S.add((b, int(s)))
                # candidates = children of the parent's strong boxes
                cand = sorted(4 * q + k for q in parent_strong for k in range(4))
                assert sorted(wl.tolist() + sl.tolist()) == cand
            assert all((s, b) in W for (b, s) in W)
            assert all((s, b) in S for (b, s) in S)
            sh = 2 * (L - l)
            for (b, s) in W:
                cov[b << sh:(b + 1) << sh, s << sh:(s + 1) << sh] += 1
        soff, sidx = T.strong[L]
        for b in range(4 ** L):
            for s in sidx[soff[b]:soff[b + 1]]:
                cov[b, s] += 1
        assert np.all(cov == 1), "coverage not exactly once"


# ---------------------------------------------------------------- whole FMM
def pin_fmm_L0_is_direct(orc):
    """L = 0 (one box): the FMM reduces to the direct sum."""
    src = workloads.points("uniform", 300, 41)
    m = workloads.strengths(300, 42)
    T = orc.Tree(src, 0)
    p, d = T.eval(m, 10, orc.KERNEL_LOG)
    rp, rd = orc.direct(src, m)
    assert _rel(p, rp) < 1e-13 and _rel(d, rd) < 1e-13


def pin_fmm_theta_small_is_direct(orc):
    """theta -> 0 makes every pair strong: the FMM is the direct sum."""
    src = workloads.points("clusters", 500, 43)
    m = workloads.strengths(500, 44)
    T = orc.Tree(src, 2, theta=1e-9)
    assert sum(len(T.weak[l][1]) for l in range(3)) == 0
    p, d = T.eval(m, 5, orc.KERNEL_LOG)
    rp, rd = orc.direct(src, m)
    assert _rel(p, rp) < 1e-13 and _rel(d, rd) < 1e-13


def pin_fmm_converges(orc):
    """The FMM converges to the direct sum geometrically in p (both kernels,
    separate targets; Phi against the branch-consistent direct sum)."""
    src = workloads.points("uniform", 3000, 45)
    tgt = workloads.points("uniform", 800, 46)
    m = workloads.strengths(3000, 47)
    T = orc.Tree(src, 3, tgt=tgt)
    _, rd = orc.direct(src, m, tgt=tgt)
    rp = T.direct_branch(m, np.arange(800))
    last = None
    for p in (6, 12, 18, 24):
        ph, dh = T.eval(m, p, orc.KERNEL_LOG)
        _, dh2 = T.eval(m, p, orc.KERNEL_HARMONIC)
        e = max(_rel(dh, rd), _rel(dh2, rd), _rel(ph, rp))
        if last is not None:
            assert e < last * 0.1, (p, e, last)
        last = e
    assert last < 1e-9


def pin_operating_point(orc):
    """Sec. 5.1: p = 17 with theta = 1/2 gives TOL of about 1e-6, where TOL is the
    pointwise relative error max_i |Phi_FMM - Phi_exact| / |Phi_exact| (harmonic
    potential, uniform points, N_d = 40).  Pinned within a factor 10 either way."""
    src = workloads.points("uniform", 10_000, 1)
    m = workloads.strengths(10_000, 101)
    L = orc.nlevels(10_000, 40)
    T = orc.Tree(src, L)
    _, d = T.eval(m, 17, orc.KERNEL_HARMONIC)
    _, rd = orc.direct(src, m, kernel=orc.KERNEL_HARMONIC)
    tol = float(np.max(np.abs(d - rd) / np.abs(rd)))
    assert 1e-7 <= tol <= 1e-5, tol


def pin_branch(orc):
    """The branch-consistent direct sum equals the principal direct sum up to
    2 pi i (integer combinations of the strengths): with real strengths its
    real part equals the principal one, and with integer strengths the
    imaginary difference is a multiple of 2 pi."""
    src = workloads.points("uniform", 1200, 48)
    T = orc.Tree(src, 3)
    sel = np.arange(0, 1200, 7)
    mr = workloads.strengths(1200, 49).real.astype(complex)
    pb = T.direct_branch(mr, sel)
    pp, _ = orc.direct(src, mr, tsel=sel)
    assert _rel(pb.real, pp.real) < 1e-12
    mi = np.round(workloads.strengths(1200, 50).real * 3).astype(complex)
    pb = T.direct_branch(mi, sel)
    pp, _ = orc.direct(src, mi, tsel=sel)
    k = (pb.imag - pp.imag) / (2 * np.pi)
    assert np.all(np.abs(k - np.round(k)) < 1e-9)
    assert np.any(np.round(k) != 0), "no cut crossing exercised"


def pin_fmm_lattice_ties(orc):
    """Points on a lattice share coordinates (ties in every split, pairs with
    equal x or equal y) and some targets coincide with sources (excluded from
    the sums by eq. (poteval)): the FMM still converges to the direct sum."""
    k = 24
    g = (np.arange(k)[:, None] + 1j * np.arange(k)[None, :]).ravel() / k
    m = workloads.strengths(g.size, 51)
    tgt = np.concatenate([g[::5], workloads.points("uniform", 100, 52)])
    for tg in (None, tgt):
        T = orc.Tree(g, 2, tgt=tg)
        _, d = T.eval(m, 30, orc.KERNEL_HARMONIC)
        _, rd = orc.direct(g, m, tgt=tg, kernel=orc.KERNEL_HARMONIC)
        assert _rel(d, rd) < 1e-10, _rel(d, rd)


def pin_p2l_near_field(orc):
    """P2L of sources outside the disc |z - c| <= rT, evaluated inside it,
    equals the direct sum within the truncated-series bound: with
    q = rT / min|x - c|, the harmonic tail is at most sum|m| q^(p+1) /
    (min|x-c| (1-q)) and the log tail sum|m| q^(p+1) / ((p+1)(1-q))."""
    x, m = _cluster(13, n=25, c=0.8 + 0.7j, rad=0.1)
    c, rT = 0.3 + 0.2j, 0.1
    dmin = float(np.min(np.abs(x - c)))
    q = rT / dmin
    am = float(np.sum(np.abs(m)))
    zs = c + rT * np.exp(1j * np.linspace(0.3, 6.0, 7))
    for p in (5, 11, 19):
        bh = orc.p2l(orc.KERNEL_HARMONIC, p, c, x, m)
        bl = orc.p2l(orc.KERNEL_LOG, p, c, x, m)
        for z in zs:
            vh, _ = orc.eval_local(p, bh, c, z)
            ref_d = np.sum(m / (z - x))
            assert abs(vh - ref_d) <= 1.01 * am * q ** (p + 1) / (dmin * (1 - q)) + 1e-14 * abs(ref_d)
            vl, dl = orc.eval_local(p, bl, c, z)
            ref_p = np.sum(m * np.log(z - x))
            assert abs(vl - ref_p) <= 1.01 * am * q ** (p + 1) / ((p + 1) * (1 - q)) + 1e-13 * abs(ref_p)
            assert abs(dl - ref_d) <= 1.01 * am * (p + 2) * q ** (p + 1) / (dmin * (1 - q) ** 2) + 1e-13 * abs(ref_d)


def pin_swap_lists(orc):
    """Leaf-level swapped criterion: M2P and P2L pairs pass r + theta R <= theta d,
    M2P has the larger target box, the two lists are mirror images, P2P pairs
    fail both criteria, and every leaf pair is still handled exactly once."""
    for dist, n, L in (("clusters", 4000, 4), ("spiral", 3000, 3)):
        src = workloads.points(dist, n, 53)
        T = orc.Tree(src, L, swap=True)
        cen = T.centre[T.boxes(L)]
        rad = T.radius[T.boxes(L)]
        moff, midx = T.m2p
        poff, pidx = T.p2l
        soff, sidx = T.strong[L]
        M = set()
        P = set()
        cov = np.zeros((4 ** L, 4 ** L), np.int64)
        for b in range(4 ** L):
            for s in midx[moff[b]:moff[b + 1]]:
                d = abs(cen[b] - cen[s])
                assert rad[b] > rad[s] and min(rad[b], rad[s]) + 0.5 * max(rad[b], rad[s]) <= 0.5 * d
                M.add((b, int(s)))
                cov[b, s] += 1
            for s in pidx[poff[b]:poff[b + 1]]:
                d = abs(cen[b] - cen[s])
                assert rad[b] < rad[s] and min(rad[b], rad[s]) + 0.5 * max(rad[b], rad[s]) <= 0.5 * d
                P.add((b, int(s)))
                cov[b, s] += 1
            for s in sidx[soff[b]:soff[b + 1]]:
                d = abs(cen[b] - cen[s])
                assert s == b or not (min(rad[b], rad[s]) + 0.5 * max(rad[b], rad[s]) <= 0.5 * d)
                cov[b, s] += 1
        assert len(M) > 0, "no swapped pair exercised"
        assert M == {(s, b) for (b, s) in P}
        for l in range(1, L + 1):
            woff, widx = T.weak[l]
            sh = 2 * (L - l)
            for b in range(4 ** l):
                for s in widx[woff[b]:woff[b + 1]]:
                    cov[b << sh:(b + 1) << sh, s << sh:(s + 1) << sh] += 1
        assert np.all(cov == 1)


def pin_fmm_swap_converges(orc):
    """With the swapped criterion the FMM still converges geometrically to the
    direct sum (Phi against the branch-consistent sum, which follows Arg(y - c_s)
    for M2P pairs and Arg(c_t - x) for P2L pairs)."""
    src = workloads.points("clusters", 3000, 54)
    m = workloads.strengths(3000, 55)
    T = orc.Tree(src, 3, swap=True)
    assert len(T.m2p[1]) > 0
    _, rd = orc.direct(src, m)
    sel = np.arange(0, 3000, 3)
    rp = T.direct_branch(m, sel)
    last = None
    for p in (6, 12, 18, 24):
        ph, dh = T.eval(m, p, orc.KERNEL_LOG)
        _, dh2 = T.eval(m, p, orc.KERNEL_HARMONIC)
        e = max(_rel(dh, rd), _rel(dh2, rd), _rel(ph[sel], rp))
        if last is not None:
            assert e < last * 0.2, (p, e, last)
        last = e
    assert last < 1e-8



# ------------------------------------------------------- per-pair orders
def pin_pair_err_point_source(orc):
    """Closed forms of the truncation bound e_q for a point source at the
    source centre.  Harmonic: a_1 = m only, so b_l = m (-1)^l rho^{-(l+1)}
    exactly and truncation at q drops rows l > q:
        e_q = |m| / |rho| sum_{l=q+1..P} (rT/|rho|)^l.
    Log: a_0 = m only, b_l = -m (-w/rho)^l / l, so
        e_q = |m| sum_{l=q+1..P} (rT/|rho|)^l / l."""
    P, m, rho, rT = 24, 0.7 - 1.3j, 2.0 + 1.5j, 0.6
    x = rT / abs(rho)
    a = np.zeros(P + 1, complex)
    a[1] = m
    e = orc.pair_err(P, a, rho, rT, 0, P)
    for q in range(1, P + 1):
        ref = abs(m) / abs(rho) * sum(x ** l for l in range(q + 1, P + 1))
        assert abs(e[q] - ref) <= 1e-13 * abs(m) / abs(rho), (q, e[q], ref)
    a = np.zeros(P + 1, complex)
    a[0] = m
    e = orc.pair_err(P, a, rho, rT, 0, P)
    for q in range(0, P + 1):
        ref = abs(m) * sum(x ** l / l for l in range(q + 1, P + 1))
        assert abs(e[q] - ref) <= 1e-13 * abs(m), (q, e[q], ref)


def pin_pair_err_bounds_error(orc):
    """e_q bounds the actual error of the truncated pair on the target disc:
    for a cluster's multipole (order P), the local expansion of the pair
    truncated at q differs from the one at P by at most e_q at every z with
    |z - c_T| <= rT, and the bound is not loose by more than a few powers."""
    P = 30
    xs, ms = _cluster(3, n=25, c=0.0, rad=0.1)
    cS, cT, rT = 0.0, 0.9 + 0.4j, 0.12
    for kernel in (orc.KERNEL_HARMONIC, orc.KERNEL_LOG):
        a = orc.p2m(kernel, P, cS, xs, ms)
        bP = orc.m2l(P, a, cT - cS)
        e = orc.pair_err(P, a, cT - cS, rT, 2, 20)
        zs = cT + rT * np.exp(2j * np.pi * np.arange(64) / 64)
        for q in range(2, 21):
            bq = np.zeros(P + 1, complex)
            bq[:q + 1] = orc.m2l(q, a[:q + 1], cT - cS)
            err = max(abs(orc.eval_local(P, bq - bP, cT, z)[0]) for z in zs)
            assert err <= e[q - 2] * (1 + 1e-9) + 1e-300, (kernel, q, err, e[q - 2])
            assert err >= e[q - 2] * 1e-3, (kernel, q, err, e[q - 2])


def pin_labels_budget(orc):
    """Labels: the budget of box T is tol min_{y in T} |val(y)| / |weak(T)|
    (recomputed here from the tree's targets and lists), and the label is the
    smallest q in [qmin, qmax] with e_q <= budget (else qmax)."""
    n = 3000
    src = workloads.points("clusters", n, 21)
    m = workloads.strengths(n, 22)
    T = orc.Tree(src, 3)
    P, tol, qmin, qmax = 24, 1e-6, 4, 20
    _, dphi, A, _ = T.eval(m, P, orc.KERNEL_HARMONIC, want_coeffs=True)
    lab, err, bud = T.labels(A, P, dphi, tol, qmin, qmax)
    lv, tb, sb = T.weak_pairs()
    assert lab.size == lv.size == T.n_weak() > 0
    k = 0
    for l in range(1, T.L + 1):
        off, idx = T.weak[l]
        st = T.starts(l, targets=True)
        for b in range(4 ** l):
            nw = int(off[b + 1] - off[b])
            if nw == 0:
                continue
            tg = T.tperm[st[b]:st[b + 1]]
            ref = tol * np.abs(dphi[tg]).min() / nw
            for e in range(nw):
                assert abs(bud[k] - ref) <= 4.5e-16 * ref, (l, b, bud[k], ref)
                ok = np.nonzero(err[k] <= bud[k])[0]
                want = qmin + ok[0] if ok.size else qmax
                assert lab[k] == want
                # e_q of the pair equals pair_err from the multipole directly
                g, gs = orc.box_offset(l) + b, orc.box_offset(l) + int(idx[off[b] + e])
                e2 = orc.pair_err(P, A[gs], T.centre[g] - T.centre[gs], T.radius[g], qmin, qmax)
                assert np.array_equal(e2, err[k])
                k += 1
    assert k == lab.size


def pin_orders_uniform(orc):
    """Every pair at order q with storage p > q equals the plain FMM at p = q
    (without the swapped criterion: P2M/M2M coefficients up to q do not depend
    on p, the local expansions carry zeros above q).  Every pair at p equals
    the plain FMM at p."""
    n = 4000
    src = workloads.points("clusters", n, 23)
    m = workloads.strengths(n, 24)
    T = orc.Tree(src, 3)
    for kernel in (orc.KERNEL_HARMONIC, orc.KERNEL_LOG):
        for q in (6, 11):
            got = T.eval(m, 20, kernel, orders=np.full(T.n_weak(), q, np.uint8))
            ref = T.eval(m, q, kernel)
            assert _rel(got[1], ref[1]) < 1e-13
            if kernel == orc.KERNEL_LOG:
                assert _rel(got[0], ref[0]) < 1e-13
        got = T.eval(m, 20, kernel, orders=np.full(T.n_weak(), 20, np.uint8))
        ref = T.eval(m, 20, kernel)
        assert np.array_equal(got[1], ref[1])


def pin_orders_per_pair(orc):
    """Per-pair orders reach the right pairs: the local expansions of a small
    tree assembled here pair by pair (orc.m2l at each pair's order, then L2L
    down the levels) equal the oracle's."""
    n = 3000
    src = workloads.points("clusters", n, 25)
    m = workloads.strengths(n, 26)
    T = orc.Tree(src, 3)
    assert int(T.weak[2][0][-1]) > 0 and int(T.weak[3][0][-1]) > 0
    p = 14
    rng = np.random.default_rng(27)
    q = rng.integers(1, p + 1, T.n_weak()).astype(np.uint8)
    _, _, A, B = T.eval(m, p, orc.KERNEL_LOG, want_coeffs=True, orders=q)
    Bref = np.zeros_like(B)
    k = 0
    for l in range(1, T.L + 1):
        off, idx = T.weak[l]
        for b in range(4 ** l):
            g = orc.box_offset(l) + b
            par = orc.box_offset(l - 1) + b // 4
            if l > 1:
                Bref[g] += orc.l2l(p, Bref[par], T.centre[g] - T.centre[par])
            for e in range(off[b], off[b + 1]):
                gs = orc.box_offset(l) + int(idx[e])
                qq = int(q[k])
                Bref[g, :qq + 1] += orc.m2l(qq, A[gs, :qq + 1], T.centre[g] - T.centre[gs])
                k += 1
    leaves = slice(orc.box_offset(T.L), orc.box_offset(T.L + 1))
    assert k == q.size
    assert _rel(B[leaves], Bref[leaves]) < 1e-13


def pin_features_invariants(orc):
    """The order features (oracle/porder.py): f2 = f0 + f1; the shares
    10^f6 of one target box sum to 1; 10^f7 is the weak count; f3 = l/L;
    f5 <= 0; and doubling every coordinate (exact in floating point) leaves
    every feature unchanged (the coefficients are scaled by the box radii)."""
    from oracle import porder
    n = 4000
    src = workloads.points("clusters", n, 28)
    m = workloads.strengths(n, 29)
    T = orc.Tree(src, 3)
    p = 20
    for kernel in (orc.KERNEL_HARMONIC, orc.KERNEL_LOG):
        A = T.eval(m, p, kernel, want_coeffs=True)[2]
        F = porder.features(T, A, p)
        lv, tb, sb = T.weak_pairs()
        assert np.allclose(F[:, 2], F[:, 0] + F[:, 1], rtol=1e-15, atol=0)
        assert np.array_equal(F[:, 3], lv / T.L)
        assert np.all(F[:, 5] <= 1e-15)
        key = lv * 4 ** T.L + tb
        share = np.zeros(key.max() + 1)
        np.add.at(share, key, 10.0 ** F[:, 6])
        cnt = np.bincount(key)
        nz = cnt > 0
        assert np.allclose(share[nz], 1.0, rtol=1e-13)
        assert np.array_equal(np.rint(10.0 ** F[:, 7]).astype(int), cnt[key])
        T2 = orc.Tree(2.0 * src, 3)
        A2 = T2.eval(m, p, kernel, want_coeffs=True)[2]
        F2 = porder.features(T2, A2, p)
        assert np.allclose(F2, F, rtol=1e-12, atol=1e-12)
    # the radius scaling matters: unscaled coefficients change under doubling
    assert not np.allclose(np.abs(A2[1:, 3]) / np.abs(A[1:, 3]).clip(1e-300), 1.0)


class _HandTree:
    """Hand-set geometry and weak pairs in the interface porder.features
    reads (L, radius, centre, weak_pairs())."""

    def __init__(self, L, radius, centre, pairs):
        self.L = L
        self.radius = radius
        self.centre = centre
        self._pairs = pairs

    def weak_pairs(self):
        lv, tb, sb = (np.array(c, np.int64) for c in zip(*self._pairs))
        return lv, tb, sb


def pin_features_closed_form(orc):
    """Every order feature against its closed form.  Geometry and weak pairs
    are set by hand (one leaf of zero radius, so its coefficients are scaled
    by the floor 2^-20 rho_root); the multipoles are geometric, a_k = c t^k,
    so |a_k| / sigma^k = |c| r^k with r = |t| / sigma and the coefficient
    norms are finite geometric sums:
      n1   = |c| (1 - r^(K+1)) / (1 - r)                 (k = 0..K)
      tail = |c| (r^(floor(K/2)+1) - r^(K+1)) / (1 - r)   (k > K/2)
    f4 = log10(n1_S / n1_root), f5 = log10(tail_S / n1_S), f6 =
    log10(n1_S / sum over weak(T) of n1), f7 = log10 |weak(T)|, f0..f3 the
    ratios of radii and distance and l / L.  K = min(p, 20): p = 24 and an
    odd K = 15 are both checked."""
    from oracle import porder
    rng = np.random.default_rng(31)
    L = 2
    nb = orc.box_offset(L + 1)
    radius = rng.uniform(0.02, 0.3, nb)
    radius[0] = 0.9
    radius[orc.box_offset(2) + 6] = 0.0          # a leaf of coincident points
    centre = rng.uniform(0, 1, nb) + 1j * rng.uniform(0, 1, nb)
    pairs = [(1, 0, 3), (1, 3, 0), (1, 1, 2)]
    # level 2: target boxes with 1, 2, 3 and 5 weak sources (zero-radius leaf among them)
    for t, srcs in ((0, (9,)), (5, (6, 14)), (6, (0, 5, 12)), (11, (1, 2, 6, 7, 15))):
        pairs += [(2, t, s) for s in srcs]
    T = _HandTree(L, radius, centre, pairs)
    sig = np.maximum(radius, radius[0] * 2.0 ** -20)
    c = rng.uniform(0.5, 2.0, nb) * np.exp(2j * np.pi * rng.random(nb))
    r = rng.uniform(0.15, 0.85, nb)
    t = r * sig * np.exp(2j * np.pi * rng.random(nb))
    for p in (24, 15):
        K = min(p, porder.FEAT_K)
        A = c[:, None] * t[:, None] ** np.arange(p + 1)[None, :]
        n1 = np.abs(c) * (1 - r ** (K + 1)) / (1 - r)
        tail = np.abs(c) * (r ** (K // 2 + 1) - r ** (K + 1)) / (1 - r)
        F = porder.features(T, A, p)
        lv, tb, sb = T.weak_pairs()
        gT = np.array([orc.box_offset(int(l)) for l in lv]) + tb
        gS = np.array([orc.box_offset(int(l)) for l in lv]) + sb
        d = np.abs(centre[gT] - centre[gS])
        den = {}
        cnt = {}
        for g_t, g_s in zip(gT, gS):
            den[g_t] = den.get(g_t, 0.0) + n1[g_s]
            cnt[g_t] = cnt.get(g_t, 0) + 1
        ref = np.empty_like(F)
        ref[:, 0] = radius[gS] / d
        ref[:, 1] = radius[gT] / d
        ref[:, 2] = (radius[gS] + radius[gT]) / d
        ref[:, 3] = lv / L
        ref[:, 4] = np.log10(n1[gS] / n1[0])
        ref[:, 5] = np.log10(tail[gS] / n1[gS])
        ref[:, 6] = np.log10(n1[gS] / np.array([den[g] for g in gT]))
        ref[:, 7] = np.log10(np.array([cnt[g] for g in gT], np.float64))
        assert np.allclose(F, ref, rtol=1e-12, atol=1e-12), (p, np.max(np.abs(F - ref), axis=0))


def _mlp_problem(seed, n=200):
    from oracle import porder
    rng = np.random.default_rng(seed)
    w = np.zeros(porder.MODEL_FLOATS)
    w[:porder.NPARAM] = rng.normal(0, 0.5, porder.NPARAM)
    o = porder.NPARAM
    w[o:o + 8] = rng.normal(0, 1, 8)               # mu
    w[o + 8:o + 16] = rng.uniform(0.5, 2, 8)       # isd
    w[o + 16:o + 24] = -1e30                       # lo
    w[o + 24:o + 32] = 1e30                        # hi
    F = rng.normal(0, 1, (n, 8))
    q = rng.integers(4, 30, n).astype(float)
    return w, F, q


def pin_mlp_forward_by_hand(orc):
    """A 2-unit network written out by hand: y = W2 . relu(W1 x + b1) + b2."""
    from oracle import porder
    w = np.zeros(porder.MODEL_FLOATS)
    W1 = np.zeros((32, 8))
    W1[0, 0], W1[0, 1], W1[1, 2] = 1.0, -2.0, 3.0
    w[:256] = W1.ravel()
    w[256:288][:2] = [0.5, -10.0]                  # b1
    w[288:320][:2] = [2.0, 7.0]                    # W2
    w[320] = 0.25                                  # b2
    w[321:329] = 1.0                               # mu
    w[329:337] = 0.5                               # isd
    f = np.array([[3.0, 1.0, 5.0, 0, 0, 0, 0, 0], [1.0, 1.0, 30.0, 0, 0, 0, 0, 0]])
    # x = (f - 1) / 2; unit 0: x0 - 2 x1 + 0.5; unit 1: 3 x2 - 10
    # row 0: x = (1, 0, 2): z0 = 1.5, z1 = -4 -> y = 2 * 1.5 + 0.25 = 3.25
    # row 1: x = (0, 0, 14.5): z0 = 0.5, z1 = 33.5 -> y = 1 + 234.5 + 0.25
    y = porder.forward(w, f)
    assert np.allclose(y, [3.25, 235.75], rtol=0, atol=1e-12), y


def pin_mlp_gradient(orc):
    """The hand-written back-propagation against central finite differences
    of the loss (away from the kinks of the pinball loss and of relu), for two
    quantiles."""
    from oracle import porder
    w, F, q = _mlp_problem(30)
    for tau in (0.5, 0.9):
        g = porder.grad(w, F, q, tau)
        rng = np.random.default_rng(31)
        for k in list(rng.choice(porder.NPARAM, 40, replace=False)) + [porder.NPARAM - 1, 256, 300]:
            h = 1e-6
            wp, wm = w.copy(), w.copy()
            wp[k] += h
            wm[k] -= h
            fd = (porder.loss(wp, F, q, tau) - porder.loss(wm, F, q, tau)) / (2 * h)
            assert abs(fd - g[k]) <= 1e-6 + 1e-5 * abs(fd), (tau, k, fd, g[k])


def pin_pinball_quantile(orc):
    """The pinball loss at quantile tau is minimised by the tau-quantile: for a
    constant model (W1 = W2 = 0, y = b2) the derivative in b2 changes sign at
    the empirical quantile of q; at tau = 1/2 the loss is half the mean
    absolute deviation."""
    from oracle import porder
    rng = np.random.default_rng(32)
    F = rng.normal(0, 1, (501, 8))
    q = rng.normal(10, 3, 501)
    w = np.zeros(porder.MODEL_FLOATS)
    w[329:337] = 1.0
    for tau in (0.1, 0.5, 0.98):
        qs = np.sort(q)
        k = int(np.ceil(tau * q.size)) - 1       # empirical tau-quantile
        for b2, sign in ((qs[k] - 1e-6, -1), (qs[k] + 1e-6, 1)):
            w[320] = b2
            g = porder.grad(w, F, q, tau)[porder.NPARAM - 1]
            assert np.sign(g) == sign, (tau, b2, g)
    w[320] = 9.0
    assert abs(porder.loss(w, F, q, 0.5) - 0.5 * np.mean(np.abs(q - 9.0))) < 1e-12


def pin_adam_first_step(orc):
    """Adam's first bias-corrected step moves every parameter by lr in the
    direction opposite to the sign of its gradient (for |g| >> eps)."""
    from oracle import porder
    w, F, q = _mlp_problem(33)
    g = porder.grad(w, F, q, 0.7)
    big = np.abs(g) > 1e-4
    w1, m1, v1 = porder.adam_step(w, g, np.zeros_like(g), np.zeros_like(g), 1, lr=0.01)
    d = w1[:porder.NPARAM] - w[:porder.NPARAM]
    assert np.allclose(d[big], -0.01 * np.sign(g[big]), rtol=1e-3)
    assert np.array_equal(w1[porder.NPARAM:], w[porder.NPARAM:])
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def pin_orders_decision(orc):
    """The FP32 order decision: ceil(y + delta) clamped to [4, p], equal to the
    FP64 forward pass except within 1e-4 of an integer; p wherever a feature
    leaves [lo, hi]."""
    from oracle import porder
    w, F, q = _mlp_problem(34, n=2000)
    w[:porder.NPARAM] *= 2.0
    w[320] = 12.0
    y64 = porder.forward(w, F) + 0.37
    qq, yd = porder.orders(w, F, 0.37, 20)
    ref = np.clip(np.ceil(y64), 4, 20)
    far = np.abs(y64 - np.rint(y64)) > 1e-4
    assert np.array_equal(qq[far], ref[far])
    assert 4 in qq and 20 in qq and len(np.unique(qq)) > 8
    w[porder.NPARAM + 16 + 3] = 0.5              # lo of feature 3
    qq2, _ = porder.orders(w, F, 0.37, 20)
    out = F[:, 3].astype(np.float32) < np.float32(0.5)
    assert np.all(qq2[out] == 20) and np.array_equal(qq2[~out], qq[~out])


ALL_PINS = [pin_level_rule, pin_direct_roots_of_unity, pin_direct_bruteforce, pin_p2m_far_field,
            pin_m2m_exact, pin_l2l_exact, pin_m2l_closed_forms, pin_m2l_convergence, pin_tree_hand,
            pin_tree_invariants, pin_tree_targets_on_pivot, pin_lists, pin_fmm_L0_is_direct,
            pin_fmm_theta_small_is_direct, pin_fmm_converges, pin_fmm_lattice_ties, pin_p2l_near_field, pin_swap_lists, pin_fmm_swap_converges, pin_operating_point, pin_branch,
            pin_pair_err_point_source, pin_pair_err_bounds_error, pin_labels_budget, pin_orders_uniform,
            pin_orders_per_pair, pin_features_invariants, pin_features_closed_form, pin_mlp_forward_by_hand, pin_mlp_gradient,
            pin_pinball_quantile, pin_adam_first_step, pin_orders_decision]
