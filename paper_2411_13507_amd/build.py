"""Compile the HIP library ``librbp.so`` in-tree for gfx950.

``python -m paper_2411_13507_amd.build`` (or ``build()``) always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbp.so")
SOURCES = ["rbp_kernels.hip", "rbp_kernels_var.hip", "rbp_chain.hip", "rbp_cut.hip", "rbp_graph.hip", "rbp_mpc.hip", "rbp_api.cpp"]
HEADERS = ["rbp_consts.hpp", "rbp_internal.hpp", "rbp_segment.hpp", "rbp_wave.hpp"]

# device-code flags: gfx950 only; packed FP32 instructions disabled (the
# compiler would otherwise form v_pk_* FP32 ops from scalar code)
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librbp.so)")


RESOURCES = os.path.join(HERE, "librbp.resources.tsv")


def _resource_table(remarks: str) -> str:
    """Kernel name, VGPRs, SGPRs, scratch bytes per lane, LDS bytes and
    occupancy from the compiler's kernel-resource-usage remarks."""
    keys = {"VGPRs": "vgpr", "TotalSGPRs": "sgpr", "ScratchSize [bytes/lane]": "scratch",
            "LDS Size [bytes/block]": "lds", "Occupancy [waves/SIMD]": "occupancy"}
    rows, cur = [], None
    for line in remarks.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split(" [-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = {"kernel": body.split(":", 1)[1].strip()}
            rows.append(cur)
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            if k.strip() in keys:
                cur[keys[k.strip()]] = v.strip()
    cols = ["kernel", "vgpr", "sgpr", "scratch", "lds", "occupancy"]
    return "\n".join(["\t".join(cols)] + ["\t".join(r.get(c, "") for c in cols) for r in rows]) + "\n"


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 (one compiler process per source, in
    parallel) and link ``librbp.so``; returns its path.  The compiler's
    per-kernel resource usage (registers, scratch, occupancy) is written
    beside it."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc(), *HIP_FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", "-o", obj,
               os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(compile_one, SOURCES))
    remarks = []
    for (obj, res), src in zip(results, SOURCES):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {src} with exit code {res.returncode}")
        remarks.append(res.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc link failed with exit code {res.returncode}")
    os.replace(tmp, LIB)
    with open(RESOURCES, "w") as fh:
        fh.write(_resource_table("\n".join(remarks)))
    build_abi_check([o for o, _ in results if not o.endswith("rbp_api.cpp.o")], verbose)
    return LIB


ABI_CHECK = os.path.join(HERE, "abi_asan_check")
ABI_DRIVER = os.path.join(os.path.dirname(HERE), "tests", "abi_asan_driver.cpp")


def build_abi_check(device_objs, verbose: bool = False):
    """AddressSanitizer build of the library's host code (argument validation
    and set-up behind the C ABI) with the driver in tests/ that exercises it:
    both compiled by g++ with -fsanitize=address (host code only), linked with
    the library's device objects.  A GPU test runs it.  Returns its path, or
    None where no g++ is found or the driver is absent."""
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists(ABI_DRIVER):
        return None
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    objdir = os.path.join(HERE, "_build")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address",
             "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include")]
    api_o, drv_o = os.path.join(objdir, "rbp_api_asan.o"), os.path.join(objdir, "abi_asan_driver.o")
    steps = [[gxx, *flags, "-c", "-o", api_o, os.path.join(CSRC, "rbp_api.cpp")],
             [gxx, *flags, "-c", "-o", drv_o, ABI_DRIVER],
             [gxx, "-fsanitize=address", "-o", ABI_CHECK + ".tmp", drv_o, api_o, *device_objs,
              "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")]]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"AddressSanitizer build of the ABI check failed with exit code {res.returncode}")
    os.replace(ABI_CHECK + ".tmp", ABI_CHECK)
    return ABI_CHECK


if __name__ == "__main__":
    print(build(verbose=True))
