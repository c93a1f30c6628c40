"""Batched reachable-Bezier-polytope segment QPs on AMD MI355X (gfx950).

The computation lives in ``librbp.so`` (HIP kernels behind the C ABI of
``include/rbp.h``); this package only marshals arguments.  Import
``paper_2411_13507_amd.api`` for ``SegmentBatchGPU`` and
``paper_2411_13507_amd.torch_fn`` for the autograd function.
"""
from ._lib import LIB_PATH, RbpError, load  # noqa: F401

__all__ = ["LIB_PATH", "RbpError", "load"]
