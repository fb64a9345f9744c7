"""Build the HIP library libbbwadg.so in-tree for gfx950 (hipcc, parallel units)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbbwadg.so")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _rocm() -> str:
    return os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p.stderr


def build(verbose: bool = False, jobs: int | None = None, defines=(), out: str | None = None) -> str:
    """Compile every HIP unit for gfx950 and link libbbwadg.so (or `out`); returns its path.

    `defines` are extra -D options for the kernels (tuning variants)."""
    hipcc = _hipcc()
    lib = out or LIB
    build_dir = BUILD if out is None else BUILD + "_" + os.path.basename(out).replace(".so", "")
    os.makedirs(build_dir, exist_ok=True)
    units = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cmds = []
    for u in units:
        obj = os.path.join(build_dir, u.replace(".hip", ".o"))
        cmds.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *[f"-D{d}" for d in defines], "-c",
                     os.path.join(CSRC, u), "-o", obj])
    for u in sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp")):  # host code
        cmds.append([hipcc, "-x", "c++", *[c for c in COMMON if c not in ("-Xclang", "-target-feature",
                                                                           "-packed-fp32-ops")],
                     f"-I{_rocm()}/include", "-D__HIP_PLATFORM_AMD__",
                     "-c", os.path.join(CSRC, u), "-o", os.path.join(build_dir, u.replace(".cpp", ".o"))])
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for err in ex.map(_run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    objs = [c[c.index("-o") + 1] for c in cmds]
    tmp = lib + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
