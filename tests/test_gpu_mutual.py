"""The mutual near field (FMM2D_FLAG_MUTUAL): at the sources, with the
harmonic kernel in FP64, every unordered pair of near-field leaves is
evaluated once for both directions (the pair symmetry of Sec. 4).

Against the oracle FMM at equal p and lists (<= 1e-12 normwise: only the
summation order differs), against the one-sided near field, bit for bit run to
run (the reverse sums are added in a fixed order), and unchanged where the flag
does not apply (log kernel, separate targets: the one-sided kernels run).
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


CASES = [("uniform", 10_000, 4, 17), ("clusters", 20_000, 5, 20), ("spiral", 10_007, 4, 12),
         ("clusters", 200_000, 6, 20)]


@pytest.mark.parametrize("swap", [False, True])
@pytest.mark.parametrize("dist,n,L,p", CASES)
def test_mutual_matches_oracle(fmm, orc, dist, n, L, p, swap):
    src = workloads.points(dist, n, 131)
    m = workloads.strengths(n, 132)
    assert -(-n // 4 ** L) <= 64
    _, gm = fmm.eval(dev(src), dev(m), p=p, levels=L, kernel="harmonic", swap=swap, mutual=True)
    _, g1 = fmm.eval(dev(src), dev(m), p=p, levels=L, kernel="harmonic", swap=swap)
    _, rd = orc.Tree(src, L, swap=swap).eval(m, p, orc.KERNEL_HARMONIC)
    e_o, e_1 = nrm(host(gm), rd), nrm(host(gm), host(g1))
    print("%s n=%d L=%d p=%d swap=%s: vs oracle %.2e, vs one-sided %.2e" % (dist, n, L, p, swap, e_o, e_1))
    assert e_o < 1e-12 and e_1 < 1e-13
    # run to run bit for bit
    _, gm2 = fmm.eval(dev(src), dev(m), p=p, levels=L, kernel="harmonic", swap=swap, mutual=True)
    assert torch.equal(gm, gm2)


def test_mutual_ignored_where_it_does_not_apply(fmm):
    src = workloads.points("clusters", 20_000, 133)
    m = workloads.strengths(20_000, 134)
    tgt = workloads.points("uniform", 3_000, 135)
    for kw in (dict(kernel="log"), dict(kernel="harmonic", tgt=dev(tgt)), dict(kernel="harmonic", precision="mixed"),
               dict(kernel="harmonic", levels=2)):  # 2: more than 64 sources per leaf
        kw = dict(kw)
        t = kw.pop("tgt", None)
        lv = kw.pop("levels", 5)
        a = fmm.eval(dev(src), dev(m), t, p=12, levels=lv, mutual=True, **kw)
        b = fmm.eval(dev(src), dev(m), t, p=12, levels=lv, mutual=False, **kw)
        assert torch.equal(a[1], b[1]), kw
        if a[0] is not None:
            assert torch.equal(a[0], b[0])


def test_mutual_pair_capacity(fmm):
    """A workspace for fewer upper leaf pairs than the lists hold: the overflow
    is reported as FMM2D_ENOSPC and the handle evaluates again afterwards."""
    from paper_1205_4611_amd import fmm2d
    src = workloads.points("clusters", 40_000, 136)
    m = workloads.strengths(40_000, 137)
    # list_cap 128 holds the lists (about 90 weak pairs per box) but only 8 upper
    # leaf pairs per leaf, against about 10 in this cloud
    fmm.eval(dev(src), dev(m), p=12, levels=6, kernel="harmonic", list_cap=128)
    with pytest.raises(fmm2d.FMMError) as e:
        fmm.eval(dev(src), dev(m), p=12, levels=6, kernel="harmonic", mutual=True, list_cap=128)
    assert e.value.code == fmm2d.ENOSPC
    _, gm = fmm.eval(dev(src), dev(m), p=12, levels=6, kernel="harmonic", mutual=True)
    _, g1 = fmm.eval(dev(src), dev(m), p=12, levels=6, kernel="harmonic")
    assert nrm(host(gm), host(g1)) < 1e-13
