"""Compile liblbm.so for gfx950 with hipcc (in-tree; the .so travels with the repository)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")

SOURCES = ["thermo.cpp", "lbm_step.hip", "lbm_batched.hip", "lbm_adjoint.hip", "lbm_fd.hip", "lbm_aa.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
    # only the declarations of include/lbm.h are exported
    "-fvisibility=hidden", "-fvisibility-inlines-hidden",
    # no packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hip_runtime_dir() -> str:
    """Directory of the HIP runtime PyTorch loads.

    The library must share ONE HIP runtime with torch (which provides the device memory
    and streams): linking ROCm's own libamdhip64.so.7 next to torch's bundled
    libamdhip64.so would put two runtimes in the process.
    """
    import torch

    d = os.path.join(os.path.dirname(torch.__file__), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError("torch does not bundle libamdhip64.so in %s" % d)
    return d


def build(verbose: bool = False, defines=(), out: str | None = None) -> str:
    """Compile and link liblbm.so (or `out`), with optional extra -D tuning macros."""
    lib = out or LIB
    objdir = os.path.join(os.path.dirname(lib), "_build" if out is None else "_build_" + os.path.basename(lib))
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for s in SOURCES:
        o = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = [HIPCC, *FLAGS, *["-D" + d for d in defines], "-c", *lang, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
               os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(o)
    rt = _hip_runtime_dir()
    tmp = lib + ".tmp%d" % os.getpid()
    link = ["g++", "-shared", "-o", tmp, *objs, "-L" + rt, "-lamdhip64", "-Wl,--disable-new-dtags", "-Wl,-rpath," + rt, "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
