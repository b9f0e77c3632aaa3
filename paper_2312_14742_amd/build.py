"""Build step of the HIP library ``libtau1.so`` (gfx950), in-tree.

Run ``python -m paper_2312_14742_amd.build`` or call :func:`build`.  hipcc
cross-compiles for gfx950 without a GPU present.  The z-march kernels of each
(lattice, precision) pair are two translation units of their own (the
per-layout kernels, and the one-launch kernels of a batch's one-row layouts),
compiled in parallel, then linked with the host API into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtau1.so")
OBJDIR = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (hipcc flag for the device pass)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]

PAIRS = [(q, p) for q in (15, 19, 27) for p in (1, 2, 3)]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    return res.stderr


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int | None = None) -> str:
    """Compile libtau1.so every time it is called; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    extra = extra or []
    jobs = jobs or min(8, os.cpu_count() or 1)
    units = [(os.path.join(CSRC, "tau1_api.hip"), os.path.join(OBJDIR, "tau1_api.o"), [])]
    for q, p in PAIRS:
        units.append((os.path.join(CSRC, "tau1_zmarch_inst.hip"),
                      os.path.join(OBJDIR, f"tau1_zm_{q}_{p}.o"),
                      [f"-DTAU1_Q={q}", f"-DTAU1_P={p}"]))
        units.append((os.path.join(CSRC, "tau1_zmarch_rows.hip"),
                      os.path.join(OBJDIR, f"tau1_zr_{q}_{p}.o"),
                      [f"-DTAU1_Q={q}", f"-DTAU1_P={p}"]))
    cmds = [[hipcc(), *HIPCC_FLAGS, *extra, *defs, "-c", src, "-o", obj]
            for src, obj, defs in units]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        logs = list(ex.map(_run, cmds))
    if verbose:
        sys.stderr.write("".join(logs))
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o, _ in units],
          "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
