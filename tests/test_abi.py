"""The C-ABI library loads on the CPU and exports every function that
include/*.h declares; the binding's ctypes structures match the C layout (as
compiled by gcc from the same header).  No compute call: these tests need no
GPU."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    decl = re.compile(r"^[A-Za-z_][\w\s\*]*?\b(fmm2d_\w+)\s*\(", re.M)
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in decl.finditer(text):
            if not text[m.start():m.end()].lstrip().startswith(("#", "typedef")):
                names.add(m.group(1))
    return names


def test_header_declares_functions():
    names = declared_functions()
    assert "fmm2d_eval" in names and "fmm2d_mlp_grad" in names
    assert len(names) >= 19


def test_library_exports_every_declared_symbol():
    from paper_1205_4611_amd import fmm2d
    lib = ctypes.CDLL(fmm2d.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(fmm2d.EXPORTS) == declared_functions()
    fmm2d.load()  # every argtypes assignment resolves


def test_host_only_calls():
    """Entry points that touch no device: the level rule and the MLP work size."""
    from paper_1205_4611_amd import fmm2d
    lib = fmm2d.load()
    assert lib.fmm2d_nlevels(45 * 4 ** 8, 45) == 8
    assert lib.fmm2d_nlevels(0, 45) == -1
    assert lib.fmm2d_mlp_work_size(256) >= 322 * 4
    o = fmm2d.make_opts()
    assert abs(o.theta - 0.5) < 1e-15 and o.levels == -1 and o.leaf_target == 0


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "fmm2d.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("opts %zu\ntopology %zu\nstats %zu\n", sizeof(fmm2d_opts), sizeof(fmm2d_topology), sizeof(fmm2d_stats));
  F(fmm2d_opts, list_cap); F(fmm2d_opts, flags); F(fmm2d_opts, p);
  F(fmm2d_topology, perm); F(fmm2d_topology, porder); F(fmm2d_topology, local);
  F(fmm2d_stats, n_weak); F(fmm2d_stats, status); F(fmm2d_stats, p_hist);
  printf("NFEAT %d\nNPARAM %d\nMODEL %d\nK %d\nQMIN %d\nSCHEMA %d\nNPHASE %d\n", FMM2D_PORDER_NFEAT,
         FMM2D_PORDER_NPARAM, FMM2D_PORDER_MODEL_FLOATS, FMM2D_PORDER_FEAT_K, FMM2D_PORDER_QMIN,
         FMM2D_PORDER_SCHEMA, FMM2D_NPHASE);
  return 0;
}
"""


def test_struct_layout_matches_header(tmp_path):
    from paper_1205_4611_amd import fmm2d
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(out["opts"]) == ctypes.sizeof(fmm2d.Opts)
    assert int(out["topology"]) == ctypes.sizeof(fmm2d.Topology)
    assert int(out["stats"]) == ctypes.sizeof(fmm2d.Stats)
    for cls, cname in ((fmm2d.Opts, "fmm2d_opts"), (fmm2d.Topology, "fmm2d_topology"),
                       (fmm2d.Stats, "fmm2d_stats")):
        for key, off in out.items():
            if key.startswith(cname + "."):
                assert getattr(cls, key.split(".")[1]).offset == int(off), key
    assert int(out["NFEAT"]) == fmm2d.PORDER_NFEAT
    assert int(out["NPARAM"]) == fmm2d.PORDER_NPARAM
    assert int(out["MODEL"]) == fmm2d.PORDER_MODEL_FLOATS
    assert int(out["K"]) == fmm2d.PORDER_FEAT_K
    assert int(out["QMIN"]) == fmm2d.PORDER_QMIN
    assert int(out["SCHEMA"]) == fmm2d.PORDER_SCHEMA
    assert int(out["NPHASE"]) == len(fmm2d.PHASES)
    # the model size is the trainable part plus mean, 1/std, lo and hi of the features
    assert fmm2d.PORDER_NPARAM == fmm2d.PORDER_HIDDEN * (fmm2d.PORDER_NFEAT + 2) + 1
    assert fmm2d.PORDER_MODEL_FLOATS == fmm2d.PORDER_NPARAM + 4 * fmm2d.PORDER_NFEAT


def test_null_handle_and_arguments():
    """Calls without a handle (or without a device) fail with FMM2D_EINVAL and
    touch nothing; this needs no GPU."""
    from paper_1205_4611_amd import fmm2d
    lib = fmm2d.load()
    o = fmm2d.make_opts()
    b = ctypes.c_size_t()
    assert lib.fmm2d_create(None, 0) == fmm2d.EINVAL
    h = ctypes.c_void_p()
    assert lib.fmm2d_create(ctypes.byref(h), -1) == fmm2d.EINVAL and not h.value
    assert lib.fmm2d_workspace_size(None, 100, 0, ctypes.byref(o), ctypes.byref(b)) == fmm2d.EINVAL
    assert lib.fmm2d_eval(None, 100, None, None, 0, None, ctypes.byref(o), None, None, None, 0, None) == fmm2d.EINVAL
    assert lib.fmm2d_direct(None, 100, None, None, 0, None, None, 0, 1, None, None, None) == fmm2d.EINVAL
    assert lib.fmm2d_sync(None, None) == fmm2d.EINVAL
    assert lib.fmm2d_get_stats(None, None) == fmm2d.EINVAL
    assert lib.fmm2d_get_topology(None, None) == fmm2d.EINVAL
    assert lib.fmm2d_last_error(None) == b"null handle"
