"""Register and scratch budget of the built kernels, from the compiler's
resource-usage remarks that the build writes beside librbp.so.

Per-lane scratch (private memory) is spill, a dynamically indexed register
array or the frame of an out-of-line call: it turns register or LDS data into
memory traffic.  The default-shape segment kernels of degree 3-7 (and the
polish-only one of degree 8), the backward, graph-cut and graph-building and
MPC kernels must have none, nor the path kernel or the one-wavefront-per-SIMD
shape.  Stated exceptions: the degree-8 and -9 segment kernels are at the
256-VGPR limit; the two-instances-per-workgroup shape spills (it is an option
the autotuner weighs, timed with its spill); the single-launch kernels hold
every degree's code in one kernel."""
import csv
import os
import re

import pytest

from paper_2411_13507_amd import build

ALLOWED = {r"solve_kernelI[fd]Li8E": 64, r"solve_kernelI[fd]Li9E": 128,
           r"solve_kernel_shapeILi[3-9]ELb[01]ELi2ELi2": 320, r"(solve|backward)_kernel_all": 1024}


@pytest.fixture(scope="module")
def table():
    if not os.path.exists(build.RESOURCES):
        pytest.skip("library not built here")
    with open(build.RESOURCES) as fh:
        return list(csv.DictReader(fh, delimiter="\t"))


def test_every_kernel_reported(table):
    names = " ".join(r["kernel"] for r in table)
    for k in ("solve_kernel", "backward_kernel", "chain_kernel", "cut_qp_kernel", "cut_prefilter_kernel",
              "graph_pairs_kernel", "hyperplane_kernel", "mpc_kernel"):
        assert k in names, k


def test_no_scratch_outside_the_stated_kernels(table):
    for r in table:
        limit = next((v for pat, v in ALLOWED.items() if re.search(pat, r["kernel"])), 0)
        assert int(r["scratch"]) <= limit, (r["kernel"], r["scratch"])
        assert int(r["vgpr"]) <= 256
