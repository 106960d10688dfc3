"""Error contract of the C ABI (include/fmm2d.h, fmm2d_eval / fmm2d_sync),
driven through ctypes directly so that the binding's own checks do not stand
in front of the library's.

Argument errors return their code from fmm2d_eval and launch nothing; a NaN or
infinite coordinate or strength is found on the device, the evaluation runs to
completion inside its buffers, and fmm2d_sync returns FMM2D_EINVAL.  After
every error the same handle and workspace evaluate correctly again.
"""
import ctypes

import numpy as np
import pytest

from paper_1205_4611_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_4611_amd import fmm2d
    f = fmm2d.FMM2D(0)
    yield f
    f.close()


def _pts(z):
    return torch.view_as_real(torch.from_numpy(np.ascontiguousarray(z, np.complex128)).cuda()).contiguous()


def _raw_eval(f, src, m, tgt, opts, dphi, ws, ws_bytes, n_src=None, n_tgt=None):
    """fmm2d_eval with raw pointers (None passes NULL)."""
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    ns = src.shape[0] if (n_src is None and src is not None) else (n_src or 0)
    nt = (0 if tgt is None else tgt.shape[0]) if n_tgt is None else n_tgt
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return f.lib.fmm2d_eval(f.h, ns, p(src), p(m), nt, p(tgt), ctypes.byref(opts), None, p(dphi), p(ws),
                            ws_bytes, stream)


def _sync(f):
    return f.lib.fmm2d_sync(f.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _good(f, fmm2d, n=3000):
    """A correct evaluation on the handle (compared with the device direct sum)."""
    z = workloads.points("uniform", n, 91)
    m = workloads.strengths(n, 92)
    s, mm = _pts(z), _pts(m)
    _, d = f.eval(s, mm, p=20, levels=3, kernel="harmonic")
    _, r = f.direct(s, mm, kernel="harmonic")
    assert float((d - r).abs().max() / r.abs().max()) < 1e-8


def test_argument_errors_return_codes(fmm):
    from paper_1205_4611_amd import fmm2d
    n = 2000
    src = _pts(workloads.points("clusters", n, 93))
    m = _pts(workloads.strengths(n, 94))
    o = fmm2d.make_opts(p=12, levels=2, kernel="harmonic")
    need = fmm.workspace_size(n, 0, o)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    dphi = torch.empty(n, dtype=torch.complex128, device="cuda")
    assert _raw_eval(fmm, src, m, None, o, dphi, ws, need) == fmm2d.OK
    assert _sync(fmm) == fmm2d.OK
    # NULL sources, strengths, workspace; no output at all
    assert _raw_eval(fmm, None, m, None, o, dphi, ws, need, n_src=n) == fmm2d.EINVAL
    assert _raw_eval(fmm, src, None, None, o, dphi, ws, need) == fmm2d.EINVAL
    assert _raw_eval(fmm, src, m, None, o, dphi, None, need) == fmm2d.EINVAL
    assert _raw_eval(fmm, src, m, None, o, None, ws, need) == fmm2d.EINVAL
    # a workspace one byte short
    assert _raw_eval(fmm, src, m, None, o, dphi, ws, need - 1) == fmm2d.ENOSPC
    assert b"workspace" in fmm.lib.fmm2d_last_error(fmm.h)
    # sizes: no sources, more leaves than sources, separate targets of count 0
    assert _raw_eval(fmm, src, m, None, o, dphi, ws, need, n_src=0) == fmm2d.EINVAL
    o6 = fmm2d.make_opts(p=12, levels=6, kernel="harmonic")
    assert _raw_eval(fmm, src, m, None, o6, dphi, ws, need) == fmm2d.EINVAL
    assert _raw_eval(fmm, src, m, src, o, dphi, ws, need, n_tgt=0) == fmm2d.EINVAL
    torch.cuda.synchronize()
    _good(fmm, fmm2d)


@pytest.mark.parametrize("where", ["src_x_nan", "src_y_inf", "m_inf", "m_nan", "tgt_nan"])
def test_nonfinite_inputs_rejected(fmm, where):
    from paper_1205_4611_amd import fmm2d
    n, nt = 5000, 3000
    z = workloads.points("clusters", n, 95)
    m = workloads.strengths(n, 96)
    t = workloads.points("uniform", nt, 97) if where == "tgt_nan" else None
    k = 1234
    if where == "src_x_nan":
        z[k] = complex(np.nan, z[k].imag)
    elif where == "src_y_inf":
        z[k] = complex(z[k].real, np.inf)
    elif where == "m_inf":
        m[k] = complex(-np.inf, 0.0)
    elif where == "m_nan":
        m[k] = complex(0.0, np.nan)
    else:
        t[17] = complex(np.nan, np.nan)
    s, mm = _pts(z), _pts(m)
    tg = None if t is None else _pts(t)
    for swap in (False, True):
        o = fmm2d.make_opts(p=17, levels=3, kernel="harmonic", swap=swap)
        need = fmm.workspace_size(n, 0 if t is None else nt, o)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        dphi = torch.empty(n if t is None else nt, dtype=torch.complex128, device="cuda")
        assert _raw_eval(fmm, s, mm, tg, o, dphi, ws, need) == fmm2d.OK  # found on the device
        assert _sync(fmm) == fmm2d.EINVAL, where
        assert b"NaN or infinite" in fmm.lib.fmm2d_last_error(fmm.h)
        # the binding raises the same code
        with pytest.raises(fmm2d.FMMError) as e:
            fmm.eval(s, mm, tg, p=17, levels=3, kernel="harmonic", swap=swap)
        assert e.value.code == fmm2d.EINVAL
    # a finite evaluation on the same handle clears the status and is correct
    _good(fmm, fmm2d)


def test_binding_checks_shapes(fmm):
    from paper_1205_4611_amd import fmm2d
    n = 1000
    s = _pts(workloads.points("uniform", n, 98))
    m = _pts(workloads.strengths(n, 99))
    with pytest.raises(ValueError):
        fmm.eval(s, m[:-1], p=10, levels=2)
    with pytest.raises(ValueError):
        fmm.eval(s, m, p=10, levels=2, dphi=torch.empty(n - 1, dtype=torch.complex128, device="cuda"))
    with pytest.raises(TypeError):
        fmm.eval(s, m, p=10, levels=2, dphi=torch.empty(n, dtype=torch.complex64, device="cuda"))
    with pytest.raises(TypeError):
        fmm.eval(s, m, p=10, levels=2, kernel="log",
                 phi=torch.empty(2 * n, dtype=torch.complex128, device="cuda")[::2])
    with pytest.raises(ValueError):
        fmm.direct(s, m[:10])
    _good(fmm, fmm2d)
