"""Thin Python binding of libfmm2d.so (the C ABI in include/fmm2d.h).

Argument marshalling only: every step of the evaluation runs in the library's
HIP kernels.  PyTorch provides device memory (inputs, outputs, workspace) and
the current HIP stream.  Loading fails loudly when the library has not been
built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm2d.so")

OK, EINVAL, ENOSPC, EHIP, ENOMODEL = 0, -1, -2, -3, -4
KERNEL = {"log": 1, "harmonic": 2}
PRECISION = {"fp64": 0, "mixed": 1, "mixed_far": 2}
PORDER = {"fixed": 0, "learned": 1, "given": 2}
STATIC_WS_BYTES = 64 << 20  # FMM2D_STATIC_WS_BYTES: the workspace of fmm2d_eval_static
FLAG_TIMING = 1
FLAG_REQUIRE_MODEL = 2
FLAG_LEAF_SWAP = 4
FLAG_MUTUAL = 8
PHASES = ("tree", "lists", "p2m", "m2m", "porder", "m2l", "l2l", "p2l", "p2p", "near_reduce")

# learned order (see include/fmm2d.h)
PORDER_SCHEMA = 1
PORDER_NFEAT = 8
PORDER_HIDDEN = 32
PORDER_NPARAM = 321
PORDER_MODEL_FLOATS = 353
PORDER_FEAT_K = 20
PORDER_QMIN = 4

#: every symbol include/fmm2d.h declares
EXPORTS = ("fmm2d_default_opts", "fmm2d_create", "fmm2d_destroy", "fmm2d_last_error",
           "fmm2d_nlevels", "fmm2d_workspace_size", "fmm2d_eval", "fmm2d_eval_static", "fmm2d_direct",
           "fmm2d_sync", "fmm2d_get_topology", "fmm2d_get_stats", "fmm2d_get_times",
           "fmm2d_set_porder_model", "fmm2d_set_pair_orders", "fmm2d_pair_features",
           "fmm2d_pair_labels", "fmm2d_mlp_work_size", "fmm2d_mlp_forward", "fmm2d_mlp_grad",
           "fmm2d_mlp_adam")


class Opts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("tol", ctypes.c_double), ("p", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("leaf_target", ctypes.c_int32),
                ("kernel", ctypes.c_uint32), ("precision", ctypes.c_uint32),
                ("porder", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("list_cap", ctypes.c_int32)]


class Topology(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("p", ctypes.c_int32), ("n_src", ctypes.c_int64),
                ("n_tgt", ctypes.c_int64)] + [
        (n, ctypes.c_void_p) for n in ("perm", "tperm", "sstart", "tstart", "centre", "radius",
                                       "weak_off", "weak_idx", "strong_off", "strong_idx",
                                       "m2p_off", "m2p_idx", "p2l_off", "p2l_idx",
                                       "mpole", "local", "porder")]


class Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_float * 10), ("n_weak", ctypes.c_int64),
                ("n_strong", ctypes.c_int64), ("n_m2p", ctypes.c_int64), ("n_p2l", ctypes.c_int64),
                ("n_p2p_pairs", ctypes.c_int64), ("n_m2p_evals", ctypes.c_int64),
                ("n_p2l_evals", ctypes.c_int64),
                ("status", ctypes.c_int32), ("used_model", ctypes.c_int32),
                ("p_hist", ctypes.c_int64 * 65)]


MODEL_PATH = os.path.join(_HERE, "porder_model.json")


def load_porder_model(path: str = MODEL_PATH):
    """(model float32[353], delta, metadata) from a JSON file written by
    train_porder.py."""
    import json
    import numpy as np
    with open(path) as fh:
        d = json.load(fh)
    if int(d.get("schema", -1)) != PORDER_SCHEMA:
        raise ValueError("%s: unknown feature schema %r" % (path, d.get("schema")))
    w = np.asarray(d["model"], dtype=np.float32)
    if w.size != PORDER_MODEL_FLOATS:
        raise ValueError("%s: model has %d floats, expected %d" % (path, w.size, PORDER_MODEL_FLOATS))
    return w, float(d["delta"]), d


_lib = None


def load():
    """Load libfmm2d.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmm2d.so not built: run `python -m paper_1205_4611_amd.build` "
                           "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    lib.fmm2d_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.fmm2d_default_opts.restype = None
    lib.fmm2d_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.fmm2d_create.restype = ctypes.c_int
    lib.fmm2d_destroy.argtypes = [P]
    lib.fmm2d_destroy.restype = None
    lib.fmm2d_last_error.argtypes = [P]
    lib.fmm2d_last_error.restype = ctypes.c_char_p
    lib.fmm2d_nlevels.argtypes = [i64, i32]
    lib.fmm2d_nlevels.restype = ctypes.c_int
    lib.fmm2d_workspace_size.argtypes = [P, i64, i64, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)]
    lib.fmm2d_workspace_size.restype = ctypes.c_int
    lib.fmm2d_eval.argtypes = [P, i64, P, P, i64, P, ctypes.POINTER(Opts), P, P, P, ctypes.c_size_t, P]
    lib.fmm2d_eval.restype = ctypes.c_int
    lib.fmm2d_eval_static.argtypes = [P, i64, P, P, i64, P, ctypes.POINTER(Opts), P, P, P]
    lib.fmm2d_eval_static.restype = ctypes.c_int
    lib.fmm2d_direct.argtypes = [P, i64, P, P, i64, P, P, i64, u32, P, P, P]
    lib.fmm2d_direct.restype = ctypes.c_int
    lib.fmm2d_sync.argtypes = [P, P]
    lib.fmm2d_sync.restype = ctypes.c_int
    lib.fmm2d_get_topology.argtypes = [P, ctypes.POINTER(Topology)]
    lib.fmm2d_get_topology.restype = ctypes.c_int
    lib.fmm2d_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.fmm2d_get_stats.restype = ctypes.c_int
    f32 = ctypes.c_float
    lib.fmm2d_get_times.argtypes = [P, P]
    lib.fmm2d_get_times.restype = ctypes.c_int
    lib.fmm2d_set_porder_model.argtypes = [P, P, i64, u32, f32]
    lib.fmm2d_set_porder_model.restype = ctypes.c_int
    lib.fmm2d_set_pair_orders.argtypes = [P, P, i64]
    lib.fmm2d_set_pair_orders.restype = ctypes.c_int
    lib.fmm2d_pair_features.argtypes = [P, P, i64, P]
    lib.fmm2d_pair_features.restype = ctypes.c_int
    lib.fmm2d_pair_labels.argtypes = [P, P, ctypes.c_double, i32, i32, P, i64, P]
    lib.fmm2d_pair_labels.restype = ctypes.c_int
    lib.fmm2d_mlp_work_size.argtypes = [i64]
    lib.fmm2d_mlp_work_size.restype = ctypes.c_size_t
    lib.fmm2d_mlp_forward.argtypes = [P, P, P, i64, P, P]
    lib.fmm2d_mlp_forward.restype = ctypes.c_int
    lib.fmm2d_mlp_grad.argtypes = [P, P, P, P, i64, f32, P, P, P, ctypes.c_size_t, P]
    lib.fmm2d_mlp_grad.restype = ctypes.c_int
    lib.fmm2d_mlp_adam.argtypes = [P, P, P, P, P, i32, f32, f32, f32, f32, P]
    lib.fmm2d_mlp_adam.restype = ctypes.c_int
    _lib = lib
    return lib


class FMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fmm2d error %d: %s" % (code, msg))
        self.code = code


def nlevels(n: int, nd: int) -> int:
    return int(load().fmm2d_nlevels(int(n), int(nd)))


def make_opts(theta=0.5, tol=1e-6, p=0, levels=-1, leaf_target=0, kernel="log",
              precision="fp64", porder="fixed", timing=False, require_model=False,
              list_cap=0, swap=False, mutual=False) -> Opts:
    o = Opts()
    load().fmm2d_default_opts(ctypes.byref(o))
    o.theta = float(theta)
    o.tol = float(tol)
    o.p = int(p)
    o.levels = int(levels)
    o.leaf_target = int(leaf_target)
    o.kernel = KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.porder = PORDER[porder] if isinstance(porder, str) else int(porder)
    o.flags = ((FLAG_TIMING if timing else 0) | (FLAG_REQUIRE_MODEL if require_model else 0)
               | (FLAG_LEAF_SWAP if swap else 0) | (FLAG_MUTUAL if mutual else 0))
    o.list_cap = int(list_cap)
    return o


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _output(t, n, dev, name):
    """A caller-given output must be a contiguous complex128 tensor of n
    entries on dev (the library writes 16 n bytes); None allocates one."""
    if t is None:
        return torch.empty(n, dtype=torch.complex128, device=dev)
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError("%s must be a contiguous complex128 tensor" % name)
    if t.device != dev or t.numel() != n:
        raise ValueError("%s must have %d entries on %s (has %d on %s)" % (name, n, dev, t.numel(), t.device))
    return t


def _as_points(z, name):
    """complex128 [n] or float64 [n,2] CUDA tensor -> contiguous float64 [n,2]."""
    if z is None:
        return None
    if not isinstance(z, torch.Tensor) or not z.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if z.is_complex():
        z = torch.view_as_real(z.to(torch.complex128).contiguous())
    if z.dtype != torch.float64 or z.dim() != 2 or z.shape[1] != 2:
        raise TypeError("%s must be complex128 [n] or float64 [n,2]" % name)
    return z.contiguous()


class FMM2D:
    """One library handle on one device, with a reusable workspace tensor."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = int(device)
        h = ctypes.c_void_p()
        rc = self.lib.fmm2d_create(ctypes.byref(h), self.device)
        if rc != OK:
            raise FMMError(rc, "fmm2d_create failed")
        self.h = h
        self.ws = None
        self._keep = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.fmm2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        msg = self.lib.fmm2d_last_error(self.h)
        return FMMError(rc, msg.decode() if msg else "")

    def workspace_size(self, n_src, n_tgt=0, opts=None, **kw) -> int:
        o = opts if opts is not None else make_opts(**kw)
        b = ctypes.c_size_t()
        rc = self.lib.fmm2d_workspace_size(self.h, int(n_src), int(n_tgt), ctypes.byref(o), ctypes.byref(b))
        if rc != OK:
            raise self._err(rc)
        return int(b.value)

    def _workspace(self, nbytes):
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:%d" % self.device)
        return self.ws

    def eval(self, src, m, tgt=None, *, opts=None, phi=None, dphi=None, check=True, **kw):
        """Evaluate Phi, Phi' (complex128 CUDA tensors in the caller's target
        order).  Returns (phi, dphi); phi is None for the harmonic kernel.
        check=True synchronises and raises on device-side errors."""
        o = opts if opts is not None else make_opts(**kw)
        s, mm, t = self._inputs(src, m, tgt)
        ns = s.shape[0]
        nt = ns if t is None else t.shape[0]
        dev = s.device
        log = o.kernel == KERNEL["log"]
        dphi = _output(dphi, nt, dev, "dphi")
        if log:
            phi = _output(phi, nt, dev, "phi")
        nbytes = self.workspace_size(ns, 0 if t is None else nt, o)
        ws = self._workspace(nbytes)
        stream = torch.cuda.current_stream(dev).cuda_stream
        self._keep = (s, mm, t)
        rc = self.lib.fmm2d_eval(self.h, ns, _ptr(s), _ptr(mm), nt if t is not None else 0, _ptr(t),
                                 ctypes.byref(o), _ptr(phi) if log else None, _ptr(dphi), _ptr(ws),
                                 ws.numel(), ctypes.c_void_p(stream))
        if rc != OK:
            raise self._err(rc)
        if check:
            self.sync()
        return (phi if log else None), dphi

    def eval_static(self, src, m, tgt=None, *, opts=None, phi=None, dphi=None, check=True, **kw):
        """As eval, in the library's static workspace (fmm2d_eval_static):
        no workspace tensor is allocated."""
        o = opts if opts is not None else make_opts(**kw)
        s, mm, t = self._inputs(src, m, tgt)
        ns = s.shape[0]
        nt = ns if t is None else t.shape[0]
        dev = s.device
        log = o.kernel == KERNEL["log"]
        dphi = _output(dphi, nt, dev, "dphi")
        if log:
            phi = _output(phi, nt, dev, "phi")
        stream = torch.cuda.current_stream(dev).cuda_stream
        self._keep = (s, mm, t)
        rc = self.lib.fmm2d_eval_static(self.h, ns, _ptr(s), _ptr(mm), nt if t is not None else 0, _ptr(t),
                                        ctypes.byref(o), _ptr(phi) if log else None, _ptr(dphi),
                                        ctypes.c_void_p(stream))
        if rc != OK:
            raise self._err(rc)
        if check:
            self.sync()
        return (phi if log else None), dphi

    def sync(self):
        stream = torch.cuda.current_stream(torch.device("cuda", self.device)).cuda_stream
        rc = self.lib.fmm2d_sync(self.h, ctypes.c_void_p(stream))
        if rc != OK:
            raise self._err(rc)

    def _inputs(self, src, m, tgt):
        """Points and strengths as contiguous float64 [n,2] tensors on this
        handle's device, with one strength per source."""
        s = _as_points(src, "src")
        mm = _as_points(m, "m")
        t = _as_points(tgt, "tgt")
        want = torch.device("cuda", self.device)
        for x, nme in ((s, "src"), (mm, "m"), (t, "tgt")):
            if x is not None and x.device != want:
                raise ValueError("%s is on %s, the handle on %s" % (nme, x.device, want))
        if mm.shape[0] != s.shape[0]:
            raise ValueError("m has %d entries for %d sources" % (mm.shape[0], s.shape[0]))
        return s, mm, t

    def direct(self, src, m, tgt=None, tsel=None, kernel="log"):
        """Device direct sum of Phi, Phi' over all sources (optionally at the
        targets tsel, an int64 CUDA tensor).  Returns (phi, dphi)."""
        s, mm, t = self._inputs(src, m, tgt)
        ns = s.shape[0]
        nt = ns if t is None else t.shape[0]
        k = KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
        if tsel is not None:
            tsel = tsel.to(device=s.device, dtype=torch.int64).contiguous()
        nout = nt if tsel is None else tsel.numel()
        dphi = torch.empty(nout, dtype=torch.complex128, device=s.device)
        phi = torch.empty(nout, dtype=torch.complex128, device=s.device) if k == 1 else None
        stream = torch.cuda.current_stream(s.device).cuda_stream
        rc = self.lib.fmm2d_direct(self.h, ns, _ptr(s), _ptr(mm), nt, _ptr(t), _ptr(tsel),
                                   0 if tsel is None else tsel.numel(), k, _ptr(phi), _ptr(dphi),
                                   ctypes.c_void_p(stream))
        if rc != OK:
            raise self._err(rc)
        return phi, dphi

    def stats(self) -> dict:
        st = Stats()
        rc = self.lib.fmm2d_get_stats(self.h, ctypes.byref(st))
        if rc != OK:
            raise self._err(rc)
        return {"ms": {k: float(st.ms[i]) for i, k in enumerate(PHASES)}, "n_weak": st.n_weak,
                "n_strong": st.n_strong, "n_m2p": st.n_m2p, "n_p2l": st.n_p2l,
                "n_p2p_pairs": st.n_p2p_pairs, "n_m2p_evals": st.n_m2p_evals,
                "n_p2l_evals": st.n_p2l_evals, "status": st.status,
                "used_model": st.used_model, "p_hist": list(st.p_hist)}

    # ---- per-interaction orders -------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(torch.device("cuda", self.device)).cuda_stream)

    def _cuda_f32(self, t, n=None, name="tensor"):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
            raise TypeError("%s must be a float32 CUDA tensor" % name)
        if n is not None and t.numel() != n:
            raise ValueError("%s must have %d entries" % (name, n))
        return t.contiguous()

    def set_porder_model(self, model, delta: float = 0.0):
        """Load an order model (FMM2D_PORDER_MODEL_FLOATS host floats), or
        drop it with model=None."""
        import numpy as np
        if model is None:
            rc = self.lib.fmm2d_set_porder_model(self.h, None, 0, PORDER_SCHEMA, 0.0)
        else:
            w = np.ascontiguousarray(np.asarray(model, dtype=np.float32).ravel())
            rc = self.lib.fmm2d_set_porder_model(self.h, w.ctypes.data_as(ctypes.c_void_p), w.size,
                                                 PORDER_SCHEMA, float(delta))
        if rc != OK:
            raise self._err(rc)

    def set_pair_orders(self, orders):
        """Orders for porder="given" evaluations: a uint8 CUDA tensor in
        weak-list order (kept alive by this object), or None."""
        if orders is None:
            self._orders = None
            rc = self.lib.fmm2d_set_pair_orders(self.h, None, 0)
        else:
            if not isinstance(orders, torch.Tensor) or not orders.is_cuda or orders.dtype != torch.uint8:
                raise TypeError("orders must be a uint8 CUDA tensor")
            self._orders = orders.contiguous()
            rc = self.lib.fmm2d_set_pair_orders(self.h, _ptr(self._orders), self._orders.numel())
        if rc != OK:
            raise self._err(rc)

    def pair_features(self):
        """Features [n_weak, 8] (float32, CUDA) of the last evaluation."""
        n = self.stats()["n_weak"]
        feat = torch.empty((max(n, 1), PORDER_NFEAT), dtype=torch.float32, device="cuda:%d" % self.device)
        rc = self.lib.fmm2d_pair_features(self.h, _ptr(feat), n, self._stream())
        if rc != OK:
            raise self._err(rc)
        self.sync()
        return feat[:n]

    def pair_labels(self, val, tol: float, qmin: int = PORDER_QMIN, qmax: int = 30):
        """Labels (uint8 CUDA [n_weak]) of the last evaluation; val is the
        complex128 CUDA output of that evaluation (Phi for log, Phi' for
        harmonic) in the caller's target order."""
        n = self.stats()["n_weak"]
        lab = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda:%d" % self.device)
        v = torch.view_as_real(val.contiguous())
        rc = self.lib.fmm2d_pair_labels(self.h, _ptr(v), float(tol), int(qmin), int(qmax), _ptr(lab), n,
                                        self._stream())
        if rc != OK:
            raise self._err(rc)
        self.sync()
        return lab[:n]

    def mlp_forward(self, model, x):
        model = self._cuda_f32(model, PORDER_MODEL_FLOATS, "model")
        x = self._cuda_f32(x, None, "x")
        n = x.shape[0]
        y = torch.empty(max(n, 1), dtype=torch.float32, device=x.device)
        rc = self.lib.fmm2d_mlp_forward(self.h, _ptr(model), _ptr(x), n, _ptr(y), self._stream())
        if rc != OK:
            raise self._err(rc)
        return y[:n]

    def mlp_grad(self, model, x, q, tau: float, work=None):
        """(grad [321], loss [1]) of the pinball loss, float32 CUDA."""
        model = self._cuda_f32(model, PORDER_MODEL_FLOATS, "model")
        x = self._cuda_f32(x, None, "x")
        q = self._cuda_f32(q, x.shape[0], "q")
        n = x.shape[0]
        nbytes = int(self.lib.fmm2d_mlp_work_size(n))
        if work is None or work.numel() < nbytes:
            work = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        grad = torch.empty(PORDER_NPARAM, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        rc = self.lib.fmm2d_mlp_grad(self.h, _ptr(model), _ptr(x), _ptr(q), n, float(tau), _ptr(grad),
                                     _ptr(loss), _ptr(work), work.numel(), self._stream())
        if rc != OK:
            raise self._err(rc)
        return grad, loss

    def mlp_adam(self, model, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on model's trainable parameters, in place."""
        for t, nme in ((model, "model"), (grad, "grad"), (m, "m"), (v, "v")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise TypeError("%s must be a contiguous float32 CUDA tensor" % nme)
        rc = self.lib.fmm2d_mlp_adam(self.h, _ptr(model), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                     float(beta1), float(beta2), float(eps), self._stream())
        if rc != OK:
            raise self._err(rc)

    def times(self) -> dict:
        """Per-phase device milliseconds of the last evaluation (needs
        timing=True in its options); waits for it, copies nothing else."""
        ms = (ctypes.c_float * len(PHASES))()
        rc = self.lib.fmm2d_get_times(self.h, ms)
        if rc != OK:
            raise self._err(rc)
        return {k: float(ms[i]) for i, k in enumerate(PHASES)}

    def topology(self, coeffs: bool = False) -> dict:
        """Host (numpy) copies of the tree, lists (and coefficients) of the
        last evaluation, for the tests."""
        import numpy as np
        tp = Topology()
        rc = self.lib.fmm2d_get_topology(self.h, ctypes.byref(tp))
        if rc != OK:
            raise self._err(rc)
        self.sync()
        L, p = tp.levels, tp.p
        nb = (4 ** (L + 1) - 1) // 3
        nst = nb + L + 1

        def dev(ptr, n, dtype):
            n = int(n)
            if n == 0:
                return np.empty(0, dtype=dtype)
            tmp = torch.empty(n * np.dtype(dtype).itemsize, dtype=torch.uint8)
            _memcpy_d2h(tmp, ptr, tmp.numel())
            return tmp.numpy().view(dtype).copy()

        woff = dev(tp.weak_off, nst, np.int32)
        soff = dev(tp.strong_off, nst, np.int32)
        so_L = nb - 4 ** L + L  # start offset of level L
        nw = int(woff[so_L + 4 ** L])
        nsg = int(soff[so_L + 4 ** L])
        nl = 4 ** L
        moff = dev(tp.m2p_off, nl + 1, np.int32)
        poff = dev(tp.p2l_off, nl + 1, np.int32)
        out = {
            "m2p_off": moff, "m2p_idx": dev(tp.m2p_idx, int(moff[-1]), np.int32),
            "p2l_off": poff, "p2l_idx": dev(tp.p2l_idx, int(poff[-1]), np.int32),
            "levels": L, "p": p,
            "perm": dev(tp.perm, tp.n_src, np.int32),
            "tperm": dev(tp.tperm, tp.n_tgt, np.int32),
            "sstart": dev(tp.sstart, nst, np.int32),
            "tstart": dev(tp.tstart, nst, np.int32),
            "centre": dev(tp.centre, 2 * nb, np.float64).view(np.complex128),
            "radius": dev(tp.radius, nb, np.float64),
            "weak_off": woff, "weak_idx": dev(tp.weak_idx, nw, np.int32),
            "strong_off": soff, "strong_idx": dev(tp.strong_idx, nsg, np.int32),
        }
        if tp.porder:
            out["porder"] = dev(tp.porder, nw, np.uint8)
        if coeffs:
            out["mpole"] = dev(tp.mpole, 2 * nb * (p + 1), np.float64).view(np.complex128).reshape(nb, p + 1)
            out["local"] = dev(tp.local, 2 * nb * (p + 1), np.float64).view(np.complex128).reshape(nb, p + 1)
        return out


def _memcpy_d2h(host_u8: torch.Tensor, dev_ptr: int, nbytes: int):
    """Copy nbytes from a raw device address into a host uint8 tensor."""
    lib = _hip()
    rc = lib.hipMemcpy(ctypes.c_void_p(host_u8.data_ptr()), ctypes.c_void_p(dev_ptr),
                       ctypes.c_size_t(nbytes), 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError("hipMemcpy failed (%d)" % rc)


_hiplib = None


def _hip():
    global _hiplib
    if _hiplib is None:
        _hiplib = ctypes.CDLL("libamdhip64.so")
        _hiplib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hiplib.hipMemcpy.restype = ctypes.c_int
    return _hiplib
