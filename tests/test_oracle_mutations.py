"""Plant plausible mistakes in copies of the oracle's C source and check that
the pins catch every one (a pin that cannot fail pins nothing).  Mistakes are
planted in the oracle only, on the CPU."""
import os
import tempfile

import pytest

import oracle
import oracle_pins

# (name, function whose body is edited, old text, new text)
MUTATIONS = [
    ("p2m log sign", "orc_p2m", "a[k] -= mj * pw / (double)k;", "a[k] += mj * pw / (double)k;"),
    ("p2m harmonic power off by one", "orc_p2m", "{ a[k] += mj * pw; pw *= d; }", "{ pw *= d; a[k] += mj * pw; }"),
    ("m2m dropped a0 term", "orc_m2m", "cplx s = -a[0] * rp[l] / (double)l;", "cplx s = 0;"),
    ("m2m binomial index", "orc_m2m", "binom(l - 1, k - 1)", "binom(l, k - 1)"),
    ("m2m shift direction", "orc_m2m", "cplx r = rx + I * ry;", "cplx r = -(rx + I * ry);"),
    ("m2l alternating sign", "orc_m2l", "double sgn = (l & 1) ? -1.0 : 1.0;", "double sgn = 1.0;"),
    ("m2l binomial index", "orc_m2l", "binom(k + l - 1, l)", "binom(k + l, l)"),
    ("m2l log term sign", "orc_m2l", "cplx s0 = a[0] * clog(rho);", "cplx s0 = -a[0] * clog(rho);"),
    ("m2l a0/l term", "orc_m2l", "cplx s = -a[0] / (double)l;", "cplx s = 0;"),
    ("l2l binomial", "orc_l2l", "binom(j, l)", "binom(j + 1, l)"),
    ("l2l shift direction", "orc_l2l", "cplx r = rx + I * ry;", "cplx r = -(rx + I * ry);"),
    ("local derivative weight", "orc_eval_local", "(double)(l + 1) * b[l + 1]", "(double)l * b[l + 1]"),
    ("median rank", "split_set", "keyed piv = kv[n / 2];", "keyed piv = kv[(n + 1) / 2];"),
    ("split axis rule", "split_set", "(r[1] - r[0] >= r[3] - r[2]) ? 0 : 1", "(r[1] - r[0] >= r[3] - r[2]) ? 1 : 0"),
    ("target split side", "split_set", "lo[k] = !(tgt[2 * t[k] + ax] >= piv.c);", "lo[k] = !(tgt[2 * t[k] + ax] > piv.c);"),
    ("radius definition", "orc_build", "T->rad[g] = 0.5 * sqrt(w * w + h * h);", "T->rad[g] = sqrt(w * w + h * h);"),
    ("child numbering", "orc_build", "ss2[2 * j] = ss[j]; ss2[2 * j + 1] = ss[j] + nlo;",
     "ss2[2 * j + 1] = ss[j]; ss2[2 * j] = ss[j] + nlo;"),
    ("theta test uses max for both", "theta_weak", "double r = rb >= rs ? rs : rb;", "double r = rb >= rs ? rb : rs;"),
    ("lists: candidates from weak", "orc_build", "for (int64_t e = T->soff[l - 1][q]; e < T->soff[l - 1][q + 1]; ++e) {\n                int64_t s = T->sidx[l - 1][e];",
     "for (int64_t e = T->woff[l - 1][q]; e < T->woff[l - 1][q + 1]; ++e) {\n                int64_t s = T->widx[l - 1][e];"),
    ("l2l source level", "eval_impl", "int64_t g = box_off(l) + b, q = box_off(l - 1) + b / 4;",
     "int64_t g = box_off(l) + b, q = box_off(l - 1) + (b / 4 + 1) % nbox(l - 1);"),
    ("p2p coincident rule", "eval_impl", "if (xx == yx && xy == yy) continue;\n                    cplx w = (yx - xx) + I * (yy - xy);\n                    cplx mj",
     "if (xx == yx) continue;\n                    cplx w = (yx - xx) + I * (yy - xy);\n                    cplx mj"),
    ("direct sum drops imaginary part of m", "orc_direct", "cplx mj = m[2 * j] + I * m[2 * j + 1];", "cplx mj = m[2 * j];"),
    ("p2l log power sign", "orc_p2l", "b[l] -= mj * pw / (double)l;", "b[l] += mj * pw / (double)l;"),
    ("p2l harmonic power", "orc_p2l", "for (int l = 0; l <= p; ++l) { pw *= di; b[l] -= mj * pw; }",
     "for (int l = 0; l <= p; ++l) { b[l] -= mj * pw; pw *= di; }"),
    ("swap m2p/p2l roles", "orc_build", "ipush(Rr[b] > Rr[c] ? &mv : &pv, (int32_t)c);", "ipush(Rr[b] > Rr[c] ? &pv : &mv, (int32_t)c);"),
    ("swapped test uses theta on r", "theta_swapped", "return d > 0.0 && r + theta * R <= theta * d;", "return d > 0.0 && theta * r + R <= theta * d;"),
    ("level rule off by one", "orc_nlevels", "while (lhs < (__int128)5 * n)", "while (lhs <= (__int128)5 * n)"),
    ("pair error radius power", "orc_pair_err", "double eq = 0.0, rl = 1.0;", "double eq = 0.0, rl = rT;"),
    ("pair error compares with q+1", "orc_pair_err", "orc_m2l(q, a, rhox, rhoy, bq);", "orc_m2l(q + 1 <= P ? q + 1 : P, a, rhox, rhoy, bq);"),
    ("label budget from the largest value", "orc_labels", "if (v < vmin) vmin = v;", "if (v > vmin || vmin == INFINITY) vmin = v;"),
    ("label takes the largest passing order", "orc_labels", "if (eq[q - qmin] <= bud) lab = q;",
     "if (eq[q - qmin] <= bud && lab == qmax) lab = q;"),
    ("pair orders indexed per level", "eval_impl", "q = qw[qbase + e];", "q = qw[e];"),
    ("pair orders ignored", "eval_impl", "orc_m2l(q, A + 2 * P1 * s,", "orc_m2l(p, A + 2 * P1 * s,"),
]

# Mistakes planted in the numpy oracle of the per-pair order (oracle/porder.py):
# (name, old text, new text)
PY_MUTATIONS = [
    ("gradient sign", "dy = -np.where(u >= 0, tau, tau - 1.0) / n", "dy = np.where(u >= 0, tau, tau - 1.0) / n"),
    ("relu derivative", "dZ = np.outer(dy, W2) * (Z > 0)", "dZ = np.outer(dy, W2) * (Z > -1.0)"),
    ("quantile side", "return u * (tau - (u < 0))", "return u * (tau - (u > 0))"),
    ("standardisation dropped", "X = (np.asarray(F, np.float64) - mu) * isd", "X = np.asarray(F, np.float64) - mu"),
    ("radius scaling dropped", "v = np.abs(A[:, :K + 1]) / sig[:, None] ** k[None, :]", "v = np.abs(A[:, :K + 1])"),
    ("share over all pairs", "np.add.at(den, gT, n1[gS])", "den[:] = n1[gS].sum()"),
    ("f2 radius sum", "F[:, 2] = (rS + rT) / d", "F[:, 2] = np.maximum(rS, rT) / d"),
    ("order rounding", "q = np.clip(np.ceil(np.clip(yd, -1e6, 1e6)), QMIN, p)", "q = np.clip(np.rint(np.clip(yd, -1e6, 1e6)), QMIN, p)"),
    ("range fallback", "q = np.where(inr, q, p)", "q = q"),
    ("adam bias correction", "mh = m / (1 - b1 ** step)", "mh = m"),
    ("f4 normalised by the target box", "F[:, 4] = lg(n1[gS] / max(n1[0], 1e-300))",
     "F[:, 4] = lg(n1[gS] / np.maximum(n1[gT], 1e-300))"),
    ("f4 without the root norm", "F[:, 4] = lg(n1[gS] / max(n1[0], 1e-300))", "F[:, 4] = lg(n1[gS])"),
    ("f5 tail from k >= K/2", "return v.sum(axis=1), v[:, 2 * k > K].sum(axis=1)",
     "return v.sum(axis=1), v[:, 2 * k >= K].sum(axis=1)"),
    ("f5 tail not relative", "F[:, 5] = lg(tail[gS] / np.maximum(n1[gS], 1e-300))", "F[:, 5] = lg(tail[gS])"),
    ("feature order K = p", "K = min(p, FEAT_K)", "K = p"),
    ("radius floor dropped", "sig = np.maximum(radius, max(radius[0] * 2.0 ** -20, 1e-300))",
     "sig = np.maximum(radius, 1e-300)"),
]


def _mutate(src, func, old, new):
    import re
    # the definition: the name, a parameter list without ';', then '{'
    mt = re.search(r"\b%s\([^;{]*\)\s*\{" % re.escape(func), src)
    assert mt, "definition of %s not found" % func
    start = mt.start()
    body = mt.end() - 1
    end = src.index("\n}\n", body)
    seg = src[start:end]
    assert seg.count(old) >= 1, "mutation anchor not found in %s: %r" % (func, old)
    return src[:start] + seg.replace(old, new, 1) + src[end:]


@pytest.fixture(scope="module")
def variants(orc):
    src = oracle.source_text()
    d = tempfile.mkdtemp(prefix="orc_mut_")
    out = []
    for k, (name, func, old, new) in enumerate(MUTATIONS):
        text = _mutate(src, func, old, new)
        so = oracle.compile_variant(text, os.path.join(d, "mut%02d.so" % k))
        out.append((name, so))
    return out


_RUNNER = r"""
import sys
sys.path[:0] = [%r, %r]
import oracle, oracle_pins
with oracle.variant(%r):
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(oracle)
        except Exception as e:
            print("caught by", pin.__name__, type(e).__name__)
            sys.exit(3)
print("not caught")
sys.exit(0)
"""


def _caught(so):
    """Run every pin on the variant in a child process (a planted mistake may
    also crash the variant, which then counts as caught)."""
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    code = _RUNNER % (os.path.dirname(here), here, so)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    return r.returncode != 0, (r.stdout + r.stderr)[-400:]


@pytest.mark.parametrize("k", range(len(MUTATIONS)), ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(variants, k):
    name, so = variants[k]
    caught, log = _caught(so)
    assert caught, "no pin catches the planted mistake: %s\n%s" % (name, log)


_PY_RUNNER = r"""
import sys, types
sys.path[:0] = [%r, %r]
import oracle
text = open(oracle.__path__[0] + "/porder.py").read()
old, new = %r, %r
assert text.count(old) >= 1, "mutation anchor not found"
mod = types.ModuleType("oracle.porder")
exec(compile(text.replace(old, new, 1), "porder_mutant.py", "exec"), mod.__dict__)
sys.modules["oracle.porder"] = mod
oracle.porder = mod
import oracle_pins
for pin in oracle_pins.ALL_PINS:
    try:
        pin(oracle)
    except Exception as e:
        print("caught by", pin.__name__, type(e).__name__, str(e)[:200])
        sys.exit(3)
print("not caught")
sys.exit(0)
"""


@pytest.mark.parametrize("k", range(len(PY_MUTATIONS)), ids=[m[0] for m in PY_MUTATIONS])
def test_planted_mistake_in_porder_is_caught(orc, k):
    import subprocess
    import sys
    name, old, new = PY_MUTATIONS[k]
    here = os.path.dirname(os.path.abspath(__file__))
    code = _PY_RUNNER % (os.path.dirname(here), here, old, new)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert "mutation anchor not found" not in r.stderr, name
    assert r.returncode == 3, "no pin catches the planted mistake: %s\n%s" % (name, (r.stdout + r.stderr)[-400:])
