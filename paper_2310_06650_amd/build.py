"""Build the HIP library libqg.so in-tree for gfx950.

    python -m paper_2310_06650_amd.build

compiles every source under csrc/ with hipcc and links the shared library
next to this file.  Packed FP32 instructions are disabled for all device
code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqg.so")

SOURCES = ["qg_api.hip", "qg_kernels.hip", "qg_screen.hip", "qg_mlp.hip", "qg_build.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _run(cmd):
    print("+", " ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.run(cmd, check=True)


# host code checked by AddressSanitizer and UndefinedBehaviorSanitizer: on a
# hipcc line every -fsanitize= goes after -Xarch_host (device code is built
# as usual); the C++ file is built by clang++ itself
SANITIZE = ["-fsanitize=address", "-fsanitize=undefined"]
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++")
SANITIZED_LIB = os.path.join(HERE, "_build", "sanitized", "libqg.so")


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every source and link the library; sanitize=True builds the
    host-sanitized variant under _build/sanitized (load it with QG_LIBRARY
    and the clang ASan runtime preloaded)."""
    objdir = os.path.join(HERE, "_build", "sanitized") if sanitize else os.path.join(HERE, "_build")
    out = SANITIZED_LIB if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    host_san = [f for flag in SANITIZE for f in ("-Xarch_host", flag)]
    extra = ["-g", "-fno-omit-frame-pointer"] if sanitize else []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC, *DEVICE, *COMMON, *extra, *(host_san if sanitize else []), "-c", path,
                   "-o", obj]
        elif sanitize:
            cmd = [CLANGXX, "-x", "c++", *COMMON, *extra, *SANITIZE, "-pthread",
                   "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++", *COMMON, "-pthread", "-c", path, "-o", obj]
        _run(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if sanitize:
        link += ["-shared-libsan", *SANITIZE]
    _run(link)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
