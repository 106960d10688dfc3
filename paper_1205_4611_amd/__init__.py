"""Adaptive 2D fast multipole evaluation for AMD MI355X (gfx950).

The compute path is the C-ABI library ``libfmm2d.so`` built from ``csrc/``;
``fmm2d`` is its thin Python binding.  Importing the package loads nothing:
``from paper_1205_4611_amd import fmm2d`` loads the library and fails loudly
when it has not been built.
"""
__all__ = ["fmm2d", "workloads"]
