"""CPU oracle for the adaptive 2D FMM evaluation (Goude & Engblom, "Adaptive
fast multipole methods on the GPU").

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product.  It shares no code
with the HIP path; the two meet only in the seeded input generators.

The arithmetic lives in ``fmm2d_oracle.c`` (plain C, FP64, compiled with
-ffp-contract=off) and in ``mlp.py`` (numpy FP64).  This module only marshals
numpy arrays through ctypes.

Parity status per function (see each docstring):
  nlevels          pinned: worked example of the level rule (Sec. 5.1)
  direct           the definition itself (eqs. paireval/poteval), pinned by
                   closed forms and a brute-force cross-check
  Tree             pinned by invariants (equal-count median splits, stable
                   order, geometry) and by a hand-worked golden fixture
  lists            pinned by invariants (symmetry, theta-test, parent rule) and
                   brute-force exactly-once coverage
  p2m/m2m/m2l/l2l  pinned by exact translation identities, convergence against
                   direct evaluation and the a-priori geometric error bound
  Tree.eval        pinned: L=0 and theta->0 reduce to the direct sum; the
                   error against the direct sum falls geometrically in p
  Tree.direct_branch  pinned: equals the principal direct sum wherever no
                   branch cut is crossed; Phi' and Re Phi agree always
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm2d_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

KERNEL_LOG = 1
KERNEL_HARMONIC = 2

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def build_native(out_path: str) -> str:
    """A copy of the oracle compiled for the host it runs on (-O3
    -march=native, still IEEE FP64 without contraction): the timed CPU
    baseline.  Built where it runs, since the host may differ from the build
    machine."""
    tmp = out_path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out_path)
    return out_path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(lib):
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_nlevels.argtypes = [i64, i64]
    lib.orc_nlevels.restype = i32
    lib.orc_direct.argtypes = [i64, P, P, i64, P, P, i64, i32, P, P]
    lib.orc_direct.restype = None
    lib.orc_binom.argtypes = [i32, i32]
    lib.orc_binom.restype = f64
    lib.orc_p2m.argtypes = [i32, i32, f64, f64, i64, P, P, P]
    lib.orc_m2m.argtypes = [i32, P, f64, f64, P]
    lib.orc_m2l.argtypes = [i32, P, f64, f64, P]
    lib.orc_l2l.argtypes = [i32, P, f64, f64, P]
    lib.orc_p2l.argtypes = [i32, i32, f64, f64, i64, P, P, P]
    lib.orc_eval_multipole.argtypes = [i32, P, f64, f64, f64, f64, P, P]
    lib.orc_eval_local.argtypes = [i32, P, f64, f64, f64, f64, P, P]
    for f in ("orc_p2m", "orc_m2m", "orc_m2l", "orc_l2l", "orc_p2l", "orc_eval_multipole", "orc_eval_local"):
        getattr(lib, f).restype = None
    lib.orc_build.argtypes = [i64, P, i64, P, i32, f64, i32]
    lib.orc_build.restype = P
    lib.orc_free.argtypes = [P]
    lib.orc_free.restype = None
    lib.orc_list_len.argtypes = [P, i32, i32]
    lib.orc_list_len.restype = i64
    lib.orc_get_list.argtypes = [P, i32, i32, P, P]
    lib.orc_get_list.restype = None
    lib.orc_get_tree.argtypes = [P, P, P, P, P, P, P]
    lib.orc_get_tree.restype = None
    lib.orc_eval.argtypes = [P, P, i32, i32, P, P, P, P]
    lib.orc_eval.restype = i32
    lib.orc_direct_branch.argtypes = [P, P, P, i64, P]
    lib.orc_direct_branch.restype = i32
    lib.orc_eval_orders.argtypes = [P, P, i32, i32, P, P, P, P, P]
    lib.orc_eval_orders.restype = i32
    lib.orc_labels.argtypes = [P, P, i32, P, f64, i32, i32, P, P, P]
    lib.orc_labels.restype = i32
    lib.orc_pair_err.argtypes = [i32, P, f64, f64, f64, i32, i32, P]
    lib.orc_pair_err.restype = None
    return lib


class variant:
    """Context manager: run the wrapper on another build of the oracle
    (used by the tests that plant mistakes in copies of the C source)."""

    def __init__(self, so_path):
        self.lib = _configure(ctypes.CDLL(so_path))

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = self.lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile C source text with the oracle's flags into out_path."""
    c = out_path[:-3] + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", c, "-o", out_path, "-lm"])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _c(a, dtype):
    """Contiguous array of dtype (complex arrays become interleaved float64)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a, dtype=np.complex128).view(np.float64)
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def nlevels(n: int, nd: int) -> int:
    """Level rule, eq. (Nlevels) of Sec. 5.1: ceil(0.5 log2(5N/(8 N_d))), >= 0."""
    return int(_load().orc_nlevels(int(n), int(nd)))


def binom(n: int, k: int) -> float:
    return float(_load().orc_binom(n, k))


def direct(src, m, tgt=None, kernel=KERNEL_LOG, tsel=None):
    """Compensated FP64 direct sum of Phi and Phi' (eq. poteval; eq. paireval
    when tgt is None), skipping coincident pairs.  Inputs are complex arrays.
    Returns (phi, dphi) as complex arrays over the selected targets (phi is
    None for the harmonic kernel)."""
    lib = _load()
    s = _c(src, np.float64)
    mm = _c(m, np.float64)
    t = None if tgt is None else _c(tgt, np.float64)
    ns = s.size // 2
    nt = ns if t is None else t.size // 2
    sel = None if tsel is None else np.ascontiguousarray(tsel, dtype=np.int64)
    nout = nt if sel is None else sel.size
    phi = np.zeros(2 * nout)
    dphi = np.zeros(2 * nout)
    lib.orc_direct(ns, _p(s), _p(mm), nt, _p(t), _p(sel), 0 if sel is None else sel.size,
                   kernel, _p(phi), _p(dphi))
    dp = dphi.view(np.complex128)
    return (phi.view(np.complex128) if kernel == KERNEL_LOG else None), dp


def p2m(kernel, p, c, x, m):
    """Multipole coefficients a_0..a_p of sources x (complex) about c (eq. multipole)."""
    x = _c(x, np.float64)
    mm = _c(m, np.float64)
    a = np.zeros(2 * (p + 1))
    _load().orc_p2m(kernel, p, float(np.real(c)), float(np.imag(c)), x.size // 2, _p(x), _p(mm), _p(a))
    return a.view(np.complex128)


def m2m(p, a_child, r, out=None):
    """Shift a multipole from c_c to c_p, r = c_c - c_p (exact)."""
    a = _c(a_child, np.float64)
    o = np.zeros(2 * (p + 1)) if out is None else _c(out, np.float64).copy()
    _load().orc_m2m(p, _p(a), float(np.real(r)), float(np.imag(r)), _p(o))
    return o.view(np.complex128)


def m2l(p, a_src, rho, out=None):
    """Multipole about c_S -> local about c_T, rho = c_T - c_S."""
    a = _c(a_src, np.float64)
    o = np.zeros(2 * (p + 1)) if out is None else _c(out, np.float64).copy()
    _load().orc_m2l(p, _p(a), float(np.real(rho)), float(np.imag(rho)), _p(o))
    return o.view(np.complex128)


def p2l(kernel, p, c, x, m, out=None):
    """Local coefficients b_0..b_p about c of sources x (complex) lying outside
    the expansion disc (leaf-level swapped criterion, Sec. 2)."""
    x = _c(x, np.float64)
    mm = _c(m, np.float64)
    o = np.zeros(2 * (p + 1)) if out is None else _c(out, np.float64).copy()
    _load().orc_p2l(kernel, p, float(np.real(c)), float(np.imag(c)), x.size // 2, _p(x), _p(mm), _p(o))
    return o.view(np.complex128)


def pair_err(P, a, rho, rT, qmin, qmax):
    """e_q (q = qmin..qmax) of one M2L pair: multipole a (order P) about c_S,
    rho = c_T - c_S, target radius rT (see orc_pair_err)."""
    aa = _c(a, np.float64)
    e = np.zeros(qmax - qmin + 1)
    _load().orc_pair_err(int(P), _p(aa), rho.real, rho.imag, float(rT), int(qmin), int(qmax), _p(e))
    return e


def l2l(p, b_par, r, out=None):
    """Re-centre a local expansion from c_p to c_c, r = c_c - c_p (exact)."""
    b = _c(b_par, np.float64)
    o = np.zeros(2 * (p + 1)) if out is None else _c(out, np.float64).copy()
    _load().orc_l2l(p, _p(b), float(np.real(r)), float(np.imag(r)), _p(o))
    return o.view(np.complex128)


def eval_multipole(p, a, c, z):
    aa = _c(a, np.float64)
    v = np.zeros(2)
    d = np.zeros(2)
    _load().orc_eval_multipole(p, _p(aa), float(np.real(c)), float(np.imag(c)),
                               float(np.real(z)), float(np.imag(z)), _p(v), _p(d))
    return complex(v[0], v[1]), complex(d[0], d[1])


def eval_local(p, b, c, z):
    bb = _c(b, np.float64)
    v = np.zeros(2)
    d = np.zeros(2)
    _load().orc_eval_local(p, _p(bb), float(np.real(c)), float(np.imag(c)),
                           float(np.real(z)), float(np.imag(z)), _p(v), _p(d))
    return complex(v[0], v[1]), complex(d[0], d[1])


def box_offset(l: int) -> int:
    return (4 ** l - 1) // 3


def start_offset(l: int) -> int:
    return box_offset(l) + l


class Tree:
    """Oracle tree and interaction lists (Sec. 2 and Sec. 3.2, readings T1-T7,
    theta-criterion lists).  src/tgt are complex arrays; tgt None means the
    evaluation points are the sources.  swap=True applies the leaf-level
    swapped criterion: finest-level strong pairs that pass it become M2P
    (target box larger) or P2L (source box larger) instead of P2P."""

    def __init__(self, src, L, theta=0.5, tgt=None, swap=False):
        lib = _load()
        self._s = _c(src, np.float64)
        self._t = None if tgt is None else _c(tgt, np.float64)
        self.ns = self._s.size // 2
        self.nt = 0 if self._t is None else self._t.size // 2
        self.L = int(L)
        self.theta = float(theta)
        self._lib = lib
        self.swap = bool(swap)
        self._h = lib.orc_build(self.ns, _p(self._s), self.nt, _p(self._t), self.L, self.theta, int(self.swap))
        if not self._h:
            raise ValueError("oracle tree: invalid arguments (need 0 <= L, 4^L <= N)")
        L = self.L
        nb = box_offset(L + 1)
        self.perm = np.zeros(self.ns, np.int32)
        self.tperm = np.zeros(max(self.nt, 1), np.int32)
        self.sstart = np.zeros(start_offset(L + 1), np.int64)
        self.tstart = np.zeros(start_offset(L + 1), np.int64)
        cen = np.zeros(2 * nb)
        self.radius = np.zeros(nb)
        lib.orc_get_tree(self._h, _p(self.perm), _p(self.tperm), _p(self.sstart), _p(self.tstart),
                         _p(cen), _p(self.radius))
        self.centre = cen.view(np.complex128)
        if self.nt == 0:
            self.tperm = self.perm
            self.tstart = self.sstart
        self.weak = []
        self.strong = []

        def get(l, which):
            n = lib.orc_list_len(self._h, l, which)
            off = np.zeros(4 ** l + 1, np.int64)
            idx = np.zeros(max(n, 1), np.int32)
            lib.orc_get_list(self._h, l, which, _p(off), _p(idx))
            return off, idx[:n]

        for l in range(L + 1):
            self.weak.append(get(l, 0))
            self.strong.append(get(l, 1))
        self.m2p = get(L, 2)
        self.p2l = get(L, 3)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_free(h)
            self._h = None

    def starts(self, l, targets=False):
        a = self.tstart if targets else self.sstart
        return a[start_offset(l):start_offset(l) + 4 ** l + 1]

    def boxes(self, l):
        return slice(box_offset(l), box_offset(l + 1))

    def n_weak(self):
        return sum(int(off[-1]) for off, _ in self.weak)

    def weak_pairs(self):
        """(level, target box, source box) of every weak pair, per-level box
        numbers, in the concatenated order of levels 1..L (the order of
        per-pair orders and labels)."""
        lv, tb, sb = [], [], []
        for l in range(1, self.L + 1):
            off, idx = self.weak[l]
            cnt = np.diff(off)
            lv.append(np.full(idx.size, l, np.int64))
            tb.append(np.repeat(np.arange(4 ** l, dtype=np.int64), cnt))
            sb.append(idx.astype(np.int64))
        if not lv:
            z = np.zeros(0, np.int64)
            return z, z, z
        return np.concatenate(lv), np.concatenate(tb), np.concatenate(sb)

    def eval(self, m, p, kernel=KERNEL_LOG, want_coeffs=False, orders=None):
        """Whole FMM evaluation (Sec. 2).  Returns (phi, dphi[, A, B]) in the
        original target order; A, B are [nboxes, p+1] complex.  orders
        (optional, uint8 [n_weak], weak_pairs() order) truncates each M2L
        pair at its own order."""
        lib = self._lib
        mm = _c(m, np.float64)
        nt = self.nt or self.ns
        phi = np.zeros(2 * nt)
        dphi = np.zeros(2 * nt)
        nb = box_offset(self.L + 1)
        A = np.zeros(2 * nb * (p + 1)) if want_coeffs else None
        B = np.zeros(2 * nb * (p + 1)) if want_coeffs else None
        if orders is not None:
            q = np.ascontiguousarray(orders, dtype=np.uint8)
            if q.size != self.n_weak():
                raise ValueError("orders must have one entry per weak pair (%d)" % self.n_weak())
            rc = lib.orc_eval_orders(self._h, _p(mm), kernel, p, _p(q), _p(phi), _p(dphi), _p(A), _p(B))
        else:
            rc = lib.orc_eval(self._h, _p(mm), kernel, p, _p(phi), _p(dphi), _p(A), _p(B))
        if rc != 0:
            raise ValueError("oracle eval failed")
        out = [phi.view(np.complex128) if kernel == KERNEL_LOG else None, dphi.view(np.complex128)]
        if want_coeffs:
            out += [A.view(np.complex128).reshape(nb, p + 1), B.view(np.complex128).reshape(nb, p + 1)]
        return tuple(out)

    def labels(self, A, P, val, tol, qmin=4, qmax=30):
        """Per-pair labels from multipoles A [nboxes, P+1] of an evaluation
        at order P and the values val (original target order): returns
        (label uint8, e_q [n_weak, qmax-qmin+1], budget) in weak_pairs()
        order (see orc_labels)."""
        nw = self.n_weak()
        a = np.ascontiguousarray(A, dtype=np.complex128).view(np.float64)
        v = np.ascontiguousarray(val, dtype=np.complex128).view(np.float64)
        lab = np.zeros(max(nw, 1), np.uint8)
        err = np.zeros(max(nw, 1) * (qmax - qmin + 1))
        bud = np.zeros(max(nw, 1))
        rc = self._lib.orc_labels(self._h, _p(a), int(P), _p(v), float(tol), int(qmin), int(qmax),
                                  _p(lab), _p(err), _p(bud))
        if rc != 0:
            raise ValueError("oracle labels: bad arguments")
        return lab[:nw], err.reshape(-1, qmax - qmin + 1)[:nw], bud[:nw]

    def direct_branch(self, m, tsel):
        """Direct sum of Phi on the branch the FMM far field follows (see the
        C source).  Raises if the lists fail to cover some leaf pair."""
        lib = self._lib
        mm = _c(m, np.float64)
        sel = np.ascontiguousarray(tsel, dtype=np.int64)
        phi = np.zeros(2 * sel.size)
        rc = lib.orc_direct_branch(self._h, _p(mm), _p(sel), sel.size, _p(phi))
        if rc != 0:
            raise AssertionError("interaction lists leave %d leaf pairs uncovered" % (-rc))
        return phi.view(np.complex128)
