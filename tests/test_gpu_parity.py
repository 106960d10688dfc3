"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tree, permutation, geometry and lists: bit-exact.  Potentials: FP64 GPU FMM
against the oracle FMM at equal p and lists (<= 1e-12 normwise: only the
summation order differs), against the direct sum within the pointwise TOL of
Sec. 5.1, and the direct-sum kernel against the oracle's compensated sum.
"""
import numpy as np
import pytest

from paper_1205_4611_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(z):
    return None if z is None else torch.from_numpy(np.ascontiguousarray(z, dtype=np.complex128)).cuda()


def host(t):
    return None if t is None else t.cpu().numpy()


def nrm(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_4611_amd import fmm2d
    f = fmm2d.FMM2D(0)
    yield f
    f.close()


# ------------------------------------------------------------------ direct
def test_direct_matches_oracle(fmm, orc):
    src = workloads.points("uniform", 3000, 61)
    m = workloads.strengths(3000, 62)
    tgt = np.concatenate([workloads.points("uniform", 900, 63), src[:100]])
    for tg in (None, tgt):
        for kernel, kname in ((orc.KERNEL_LOG, "log"), (orc.KERNEL_HARMONIC, "harmonic")):
            rp, rd = orc.direct(src, m, tgt=tg, kernel=kernel)
            gp, gd = fmm.direct(dev(src), dev(m), dev(tg), kernel=kname)
            torch.cuda.synchronize()
            assert nrm(host(gd), rd) < 1e-13
            if kernel == orc.KERNEL_LOG:
                assert nrm(host(gp), rp) < 1e-13
    sel = np.array([5, 17, 2999, 0, 1234], np.int64)
    rp, rd = orc.direct(src, m, tsel=sel)
    gp, gd = fmm.direct(dev(src), dev(m), tsel=torch.from_numpy(sel).cuda())
    assert nrm(host(gd), rd) < 1e-13 and nrm(host(gp), rp) < 1e-13


# ------------------------------------------------------------------ tree
TREE_CASES = [
    # name, dist, n, L, target spec (dist, n, seed) or None
    ("uniform10k", "uniform", 10_000, 4, None),
    ("clusters20k", "clusters", 20_000, 5, None),
    ("spiral_ragged", "spiral", 10_007, 4, None),
    ("gauss10_targets", "gauss10", 6_000, 3, ("gauss10", 4_000, 71)),
    ("circle_targets", "circle", 5_000, 3, ("circle", 5_003, 72)),
    ("normal_L0", "normal", 333, 0, None),
    ("layer_L1_targets", "layer", 50, 1, ("uniform", 7, 73)),
    # deep levels with separate targets: every split runs as a global step and
    # the last ones cut tiles into hundreds of segments of a few sources
    ("dense_L5_targets", "uniform", 5_000, 5, ("uniform", 300, 75)),
    # separate targets at L = 6: the last split steps have more than 1024
    # segments, so the lo counts of both source lists and of the targets are
    # scanned in one batched set of launches
    ("clusters_L6_targets", "clusters", 20_000, 6, ("uniform", 3_000, 76)),
]


def _lattice():
    k = 24
    return (np.arange(k)[:, None] + 1j * np.arange(k)[None, :]).ravel() / k


def _case(name):
    for c in TREE_CASES:
        if c[0] == name:
            _, dist, n, L, tspec = c
            src = workloads.points(dist, n, 70)
            tgt = None if tspec is None else workloads.points(tspec[0], tspec[1], tspec[2])
            return src, tgt, L
    if name == "lattice_ties":
        g = _lattice()
        return g, np.concatenate([g[::7], workloads.points("uniform", 40, 74)]), 2
    if name in ("dense_core", "dense_core_L6"):
        # a tight core inside sparse uniform points: the boxes next to the core
        # have hundreds of strong boxes, so their children's candidate sets
        # (above 512) are shared by a workgroup in the list build
        n, frac, sig, L = (40_000, 0.9, 1e-3, 5) if name == "dense_core" else (60_000, 0.95, 3e-4, 6)
        rng = np.random.default_rng(97)
        nc = int(n * frac)
        core = (0.37 + 0.41j) + sig * (rng.standard_normal(nc) + 1j * rng.standard_normal(nc))
        return np.concatenate([core, rng.random(n - nc) + 1j * rng.random(n - nc)]), None, L
    if name == "signed_zeros":
        # -0 and +0 compare equal (ties broken by index) but the sign of a
        # zero box end reaches the centre: most zero coordinates are -0
        g = _lattice()
        flip = np.arange(g.size) % 3 != 1
        g.real[(g.real == 0) & flip] = -0.0
        g.imag[(g.imag == 0) & flip] = -0.0
        return g, None, 3
    raise KeyError(name)


def _compare_topology(orc, top, T, L):
    assert np.array_equal(top["perm"], T.perm)
    nt = T.nt or T.ns
    assert np.array_equal(top["tperm"][:nt], T.tperm[:nt])
    assert np.array_equal(top["sstart"].astype(np.int64), T.sstart)
    assert np.array_equal(top["tstart"].astype(np.int64), T.tstart)
    # geometry bit for bit
    assert np.array_equal(top["centre"].view(np.uint64), T.centre.view(np.uint64))
    assert np.array_equal(top["radius"].view(np.uint64), T.radius.view(np.uint64))
    for l in range(L + 1):
        so = orc.start_offset(l)
        nbl = 4 ** l
        for key, lists in (("weak", T.weak), ("strong", T.strong)):
            off = top[key + "_off"][so:so + nbl + 1].astype(np.int64)
            idx = top[key + "_idx"][off[0]:off[-1]]
            ro, ri = lists[l]
            assert np.array_equal(off - off[0], ro), (key, l)
            assert np.array_equal(idx, ri), (key, l)
    for key, lst in (("m2p", T.m2p), ("p2l", T.p2l)):
        off = top[key + "_off"].astype(np.int64)
        assert np.array_equal(off, lst[0]), key
        assert np.array_equal(top[key + "_idx"][:off[-1]], lst[1]), key


@pytest.mark.parametrize("swap", [False, True])
@pytest.mark.parametrize("name", [c[0] for c in TREE_CASES] + ["lattice_ties", "signed_zeros", "dense_core",
                                                               "dense_core_L6"])
def test_tree_and_lists_bitexact(fmm, orc, name, swap):
    src, tgt, L = _case(name)
    m = workloads.strengths(len(src), 75)
    fmm.eval(dev(src), dev(m), dev(tgt), p=8, levels=L, kernel="harmonic", swap=swap)
    top = fmm.topology()
    T = orc.Tree(src, L, tgt=tgt, swap=swap)
    if swap and name == "clusters20k":
        assert len(T.m2p[1]) > 0, "case does not exercise the swapped criterion"
    if name.startswith("dense_core"):
        # some box has more than 512 candidates (4 x its parent's strong count)
        assert max(4 * int(np.diff(T.strong[l][0]).max()) for l in range(L)) > 512
    _compare_topology(orc, top, T, L)


# ------------------------------------------------------------------ FMM
@pytest.mark.parametrize("kernel", ["log", "harmonic"])
@pytest.mark.parametrize("name,p,swap", [("uniform10k", 17, False), ("clusters20k", 12, False),
                                         ("gauss10_targets", 20, False), ("lattice_ties", 30, False),
                                         ("spiral_ragged", 9, False), ("clusters20k", 17, True),
                                         ("gauss10_targets", 14, True), ("spiral_ragged", 21, True),
                                         ("dense_core", 12, True)])
def test_fmm_matches_oracle_fmm(fmm, orc, name, p, swap, kernel):
    src, tgt, L = _case(name)
    m = workloads.strengths(len(src), 76)
    k = orc.KERNEL_LOG if kernel == "log" else orc.KERNEL_HARMONIC
    gp, gd = fmm.eval(dev(src), dev(m), dev(tgt), p=p, levels=L, kernel=kernel, swap=swap)
    top = fmm.topology(coeffs=True)
    T = orc.Tree(src, L, tgt=tgt, swap=swap)
    rp, rd, A, B = T.eval(m, p, k, want_coeffs=True)
    # coefficients weighted by their size on the box's disc: a_k / rho^k and
    # b_l rho^l (raw high-order coefficients carry rounding relative to terms
    # that cancel; the weighted ones measure what reaches the potential)
    kk = np.arange(p + 1)
    for l in range(L + 1):
        s = T.boxes(l)
        rho = np.maximum(T.radius[s], 1e-300)[:, None]
        assert nrm(top["mpole"][s] / rho ** kk, A[s] / rho ** kk) < 1e-12, ("multipole", l)
        if l >= 1:
            assert nrm(top["local"][s] * rho ** kk, B[s] * rho ** kk) < 1e-12, ("local", l)
    assert nrm(host(gd), rd) < 1e-12
    if kernel == "log":
        assert nrm(host(gp), rp) < 1e-12


@pytest.mark.parametrize("kernel", ["log", "harmonic"])
@pytest.mark.parametrize("p,swap", [(50, False), (64, True), (64, False)])
def test_high_orders_match_oracle(fmm, orc, p, swap, kernel):
    """Orders up to the library's maximum (64: two row tiles more than at
    p = 20 and the widest k-step bodies of the M2L kernel) against the
    oracle FMM at equal p and lists."""
    src, tgt, L = _case("clusters20k" if swap else "gauss10_targets")
    m = workloads.strengths(len(src), 87)
    k = orc.KERNEL_LOG if kernel == "log" else orc.KERNEL_HARMONIC
    gp, gd = fmm.eval(dev(src), dev(m), dev(tgt), p=p, levels=L, kernel=kernel, swap=swap)
    rp, rd = orc.Tree(src, L, tgt=tgt, swap=swap).eval(m, p, k)
    e = nrm(host(gd), rd)
    print("p=%d %s swap=%s: dphi normwise %.2e" % (p, kernel, swap, e))
    assert e < 1e-12
    if kernel == "log":
        assert nrm(host(gp), rp) < 1e-12


def test_tol_1e10_pointwise(fmm, orc):
    """TOL 1e-10 (Sec. 5.1) at the a-priori order p = ceil(log 1e-10 / log
    theta) = 34 (p = 0 with tol given): 10,000 uniform sources, Phi' pointwise
    against the compensated direct sum."""
    src = workloads.points("uniform", 10_000, 1)
    m = workloads.strengths(10_000, 101)
    L = orc.nlevels(10_000, 40)
    _, gd = fmm.eval(dev(src), dev(m), p=0, tol=1e-10, levels=L, kernel="harmonic")
    assert fmm.topology()["p"] == 34
    _, rd = orc.direct(src, m, kernel=orc.KERNEL_HARMONIC)
    e = float(np.max(np.abs(host(gd) - rd) / np.abs(rd)))
    print("TOL 1e-10 at p=34: pointwise %.2e" % e)
    assert e < 1e-10


def test_calibrated_leaf_target(fmm):
    """leaf_target 0 takes the N_d calibrated for the order in eq. (Nlevels):
    45 up to p = 26, 100 from p = 27."""
    from paper_1205_4611_amd import fmm2d
    n = 1 << 21
    src = dev(workloads.points("uniform", n, 141))
    m = dev(workloads.strengths(n, 142))
    for p, nd, L in ((20, 45, 8), (30, 100, 7)):
        fmm.eval(src, m, p=p, levels=-1, leaf_target=0, kernel="harmonic")
        assert fmm.topology()["levels"] == fmm2d.nlevels(n, nd) == L, p


def test_l0_is_direct(fmm, orc):
    src = workloads.points("clusters", 700, 77)
    m = workloads.strengths(700, 78)
    gp, gd = fmm.eval(dev(src), dev(m), p=5, levels=0, kernel="log")
    rp, rd = orc.direct(src, m)
    assert nrm(host(gd), rd) < 1e-13 and nrm(host(gp), rp) < 1e-13


def test_log_pairs_wide_range(fmm, orc):
    """The logarithm and the argument of the LOG kernel's near-field pairs
    over separations from 1 down to 1e-12, every octant, pairs on an axis
    (a zero difference of y: the principal branch puts +pi on the negative
    axis), pairs on the diagonal (|dx| = |dy|) and a geometric approach to one
    point: at L = 0 every pair is a P2P pair, so Phi and Phi' are compared
    with the oracle's direct sum, and every target's error with the sum of
    the sizes of its terms."""
    rng = np.random.default_rng(191)
    pts = [rng.uniform(0.0, 1.0, 500) + 1j * rng.uniform(0.0, 1.0, 500),   # every octant
           rng.uniform(0.1, 0.9, 300) + 0.5j,                                # dy = 0 pairs
           (lambda t: t + 1j * t)(rng.uniform(0.1, 0.9, 300)),               # |dx| = |dy|
           0.3 + 0.7j + 1e-12 * (rng.normal(size=300) + 1j * rng.normal(size=300)),
           0.6 + 0.2j + 10.0 ** (-np.arange(120) / 10.0) * np.exp(1j * rng.uniform(-np.pi, np.pi, 120))]
    src = np.concatenate(pts)
    n = len(src)
    m = workloads.strengths(n, 192)
    gp, gd = fmm.eval(dev(src), dev(m), p=5, levels=0, kernel="log")
    rp, rd = orc.direct(src, m)
    gp, gd = host(gp), host(gd)
    # the size of every target's terms: sum_j |m_j| (|Log(y - x_j)| + 1 / |y - x_j|)
    scale = np.zeros(n)
    for i0 in range(0, n, 256):
        w = src[i0:i0 + 256, None] - src[None, :]
        ok = w != 0
        lw = np.where(ok, np.log(np.where(ok, w, 1.0)), 0.0)
        iw = np.where(ok, 1.0 / np.where(ok, np.abs(w), 1.0), 0.0)
        scale[i0:i0 + 256] = (np.abs(m)[None, :] * (np.abs(lw) + iw)).sum(axis=1)
    e_p = np.max(np.abs(gp - rp) / scale)
    e_d = np.max(np.abs(gd - rd) / scale)
    print("log pairs: Phi %.2e, Phi' %.2e of the terms' size" % (e_p, e_d))
    assert e_p < 1e-14 and e_d < 1e-14
    assert nrm(gp, rp) < 1e-13 and nrm(gd, rd) < 1e-13


def test_operating_point_tol(fmm, orc):
    """10,000 uniform sources at the sources, theta 1/2, p = 17: pointwise
    relative error of Phi' about 1e-6 (TOL of Sec. 5.1), Phi against the
    branch-consistent direct sum."""
    src = workloads.points("uniform", 10_000, 1)
    m = workloads.strengths(10_000, 101)
    L = orc.nlevels(10_000, 40)
    gp, gd = fmm.eval(dev(src), dev(m), p=17, levels=L, kernel="log")
    _, rd = orc.direct(src, m, kernel=orc.KERNEL_HARMONIC)
    err_pt = float(np.max(np.abs(host(gd) - rd) / np.abs(rd)))
    assert err_pt < 2e-6, err_pt
    T = orc.Tree(src, L)
    sel = workloads.sample_indices(10_000, 500, 3)
    rb = T.direct_branch(m, sel)
    assert nrm(host(gp)[sel], rb) < 1e-8


def test_near_duplicates_harmonic(fmm, orc):
    """Point pairs 1e-12 and 1e-25 apart (the second group next to the origin,
    where such separations are representable), above the 2^-100 below which
    the FP64 harmonic near field perturbs 1/|w|^2: the FMM at the sources
    against the oracle FMM at equal p, pointwise."""
    rng = np.random.default_rng(93)
    base = workloads.points("uniform", 3000, 91)
    ang = np.exp(2j * np.pi * rng.random(300))
    near0 = 1e-20 * (rng.random(50) + 1j * rng.random(50))
    src = np.concatenate([base, base[:300] + 1e-12 * ang, near0, near0 + 1e-25 * ang[:50]])
    m = workloads.strengths(len(src), 94)
    L = orc.nlevels(len(src), 40)
    _, gd = fmm.eval(dev(src), dev(m), p=17, levels=L, kernel="harmonic")
    _, rd = orc.Tree(src, L).eval(m, 17, orc.KERNEL_HARMONIC)
    rel = np.abs(host(gd) - rd) / np.abs(rd)
    assert np.max(np.abs(rd[3000:3300])) > 1e11 and np.max(np.abs(rd[3300:])) > 1e24
    assert float(np.max(rel)) < 1e-9, float(np.max(rel))


def test_schedules_agree(fmm):
    """The timed schedule (phases in order on one stream) and the default one
    (far field on the side stream) run the same kernels on the same data:
    bit-identical outputs."""
    src = workloads.points("clusters", 40_000, 95)
    m = workloads.strengths(40_000, 96)
    for kernel in ("log", "harmonic"):
        a = fmm.eval(dev(src), dev(m), p=17, kernel=kernel, swap=True)
        b = fmm.eval(dev(src), dev(m), p=17, kernel=kernel, swap=True, timing=True)
        torch.cuda.synchronize()
        assert torch.equal(a[1], b[1])
        if kernel == "log":
            assert torch.equal(a[0], b[0])


def test_deterministic(fmm):
    src = workloads.points("clusters", 30_000, 79)
    m = workloads.strengths(30_000, 80)
    a = fmm.eval(dev(src), dev(m), p=17, kernel="log")
    b = fmm.eval(dev(src), dev(m), p=17, kernel="log")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ------------------------------------------------------------------ errors
def test_error_paths(fmm):
    from paper_1205_4611_amd import fmm2d
    src = dev(workloads.points("uniform", 100, 81))
    m = dev(workloads.strengths(100, 82))
    for kw in (dict(theta=1.5), dict(theta=0.0), dict(p=100), dict(levels=4), dict(p=0, tol=-1.0),
               dict(leaf_target=-1)):
        with pytest.raises(fmm2d.FMMError) as e:
            fmm.eval(src, m, **kw)
        assert e.value.code == fmm2d.EINVAL, kw
    # list overflow is found on the device and reported by the sync
    with pytest.raises(fmm2d.FMMError) as e:
        fmm.eval(dev(workloads.points("uniform", 5000, 83)), dev(workloads.strengths(5000, 84)),
                 levels=4, list_cap=1)
    assert e.value.code == fmm2d.ENOSPC
    # the handle still works afterwards
    fmm.eval(src, m, levels=1, p=4)


# ------------------------------------------------------------------ mixed
@pytest.mark.parametrize("kernel", ["log", "harmonic"])
@pytest.mark.parametrize("name", ["clusters20k", "gauss10_targets"])
def test_mixed_close_to_fp64(fmm, orc, name, kernel):
    """FP32 P2P and FP32 M2L (radius-scaled, MFMA) against the FP64 oracle FMM
    at the same order and lists: a check of the FP32 kernels, whose rounding
    stays near 1e-7 relative to the potential's scale (normwise).  It is not
    the TOL metric: test_mixed_meets_tol_pointwise states that one."""
    src, tgt, L = _case(name)
    m = workloads.strengths(len(src), 85)
    k = orc.KERNEL_LOG if kernel == "log" else orc.KERNEL_HARMONIC
    gp, gd = fmm.eval(dev(src), dev(m), dev(tgt), p=17, levels=L, kernel=kernel, precision="mixed")
    T = orc.Tree(src, L, tgt=tgt)
    rp, rd = T.eval(m, 17, k)
    e_d = nrm(host(gd), rd)
    print("mixed %s %s: dphi normwise %.2e" % (name, kernel, e_d))
    assert e_d < 2e-6
    if kernel == "log":
        e_p = nrm(host(gp), rp)
        print("mixed %s %s: phi normwise %.2e" % (name, kernel, e_p))
        assert e_p < 2e-6


@pytest.mark.xfail(strict=False, reason="the FP32 far field and near field round at ~1e-7 of a typical "
                   "contribution, more than 1e-6 of |Phi'| at targets where Phi' nearly cancels: the mixed path "
                   "misses TOL 1e-6 pointwise on clustered data")
@pytest.mark.parametrize("precision", ["mixed", "mixed_far"])
def test_mixed_meets_tol_pointwise(fmm, orc, precision):
    """The mixed-precision paths against the TOL 1e-6 of Sec. 5.1 in its own
    metric (pointwise relative error of Phi' against the direct sum) on
    40,000 clustered sources at p = 20."""
    src = workloads.points("clusters", 40_000, 88)
    m = workloads.strengths(40_000, 89)
    L = orc.nlevels(40_000, 45)
    _, gd = fmm.eval(dev(src), dev(m), p=20, levels=L, kernel="harmonic", swap=True, precision=precision)
    _, rd = orc.direct(src, m, kernel=orc.KERNEL_HARMONIC)
    e = float(np.max(np.abs(host(gd) - rd) / np.abs(rd)))
    print("%s: pointwise %.2e" % (precision, e))
    assert e < 1e-6


def test_heavy_boxes_match_oracle(fmm, orc):
    """A point set with a few large sparse leaves next to dense clusters, so
    that some boxes exceed the one-wave thresholds of the near field (32
    entries) and of M2L (256 weak pairs) and take the multi-wave paths."""
    src = workloads.points("clusters", 200_000, 86)
    m = workloads.strengths(200_000, 87)
    L = 6
    T = orc.Tree(src, L, swap=True)
    ne = np.diff(T.strong[L][0]) + np.diff(T.m2p[0])
    nw_max = max(int(np.diff(T.weak[l][0]).max()) for l in range(1, L + 1))
    assert ne.max() > 32 and nw_max > 256, (ne.max(), nw_max)
    for kernel, k in (("harmonic", orc.KERNEL_HARMONIC), ("log", orc.KERNEL_LOG)):
        gp, gd = fmm.eval(dev(src), dev(m), p=12, levels=L, kernel=kernel, swap=True)
        rp, rd = T.eval(m, 12, k)
        assert nrm(host(gd), rd) < 1e-12
        if k == orc.KERNEL_LOG:
            assert nrm(host(gp), rp) < 1e-12
        gp2, gd2 = fmm.eval(dev(src), dev(m), p=12, levels=L, kernel=kernel, swap=True, precision="mixed")
        assert nrm(host(gd2), rd) < 2e-6
