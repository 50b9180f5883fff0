"""Build libafm.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1109_0334_amd.build   (or build() from Python)

Every HIP translation unit is compiled with packed FP32 instructions disabled (the kernels are
written in scalar FP32/FP64 and must not be auto-vectorised into v_pk_* forms) and with
floating-point contraction limited to single expressions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libafm.so")
# the forward kernels are compiled once per force law and precision, in parallel
SOURCES = ["forward_dmt_mixed.hip", "forward_dmt_fp64.hip", "forward_kv_mixed.hip",
           "forward_kv_fp64.hip", "forward_lj_mixed.hip", "forward_lj_fp64.hip",
           "forward_hooke_mixed.hip", "forward_hooke_fp64.hip", "forward_sd_mixed.hip",
           "forward_sd_fp64.hip", "forward_none_mixed.hip", "forward_none_fp64.hip",
           "grad.hip", "api.hip", "forward.hip", "lbfgs.hip", "pso.hip", "invert.hip",
           "modes.hip", "points.hip", "noalloc.hip", "setpoint.hip"]
ARCH = os.environ.get("AFM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contract a*b + c into an fma only within one source expression, the same way in every
    # template instantiation (the default leaves the choice to the backend, which can fuse a
    # different product of a*b + c*d in two instantiations of the same code and so break the
    # bit-identity of launch shapes and kernel forms)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _stale(src: str, obj: str) -> bool:
    """An object is stale when it is older than its source, any header or this script."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src), os.path.abspath(__file__)]
    deps += [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps += [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE) if h.endswith(".h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src: str, verbose: bool, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [_hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)  # host pass does not know the feature
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile the sources and link libafm.so next to this file; returns its path.  force=False
    recompiles only objects older than their source or any header (a development shortcut)."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), SOURCES))
    tmp = LIB + ".tmp"
    r = subprocess.run([_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--incremental" not in sys.argv))
