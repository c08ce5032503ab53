"""Build libflusi.so (HIP, gfx950) in-tree with hipcc.

Each grid size is its own translation unit so the compile runs in parallel.
Usage: python -m paper_1506_06513_amd.build [--jobs J] [--sizes 64,128]
"""
from __future__ import annotations

import argparse
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflusi.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def sizes() -> list[int]:
    txt = open(os.path.join(CSRC, "sizes.def")).read()
    return [int(m) for m in re.findall(r"FLUSI_SIZE\((\d+)\)", txt)]


def boxes() -> list[tuple[int, int]]:
    """Non-cubic grids (nx, n): nx points on x, n on y and z."""
    txt = open(os.path.join(CSRC, "sizes.def")).read()
    return [(int(a), int(b)) for a, b in re.findall(r"FLUSI_BOX\((\d+),\s*(\d+)\)", txt)]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{msg}")
    return r


def build(jobs: int | None = None, out: str = LIB, verbose: bool = False) -> str:
    jobs = jobs or min(16, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="flusi_build_") as tmp:
        units = [(os.path.join(CSRC, "flusi.hip"), [], os.path.join(tmp, "flusi.o")),
                 (os.path.join(CSRC, "server.hip"), [], os.path.join(tmp, "server.o"))]
        for n in sizes():
            units.append((os.path.join(CSRC, "inst.hip"), [f"-DFLUSI_N={n}"],
                          os.path.join(tmp, f"inst_{n}.o")))
        for nx, n in boxes():
            units.append((os.path.join(CSRC, "inst.hip"), [f"-DFLUSI_NX={nx}", f"-DFLUSI_N={n}"],
                          os.path.join(tmp, f"inst_{nx}x{n}.o")))
        cmds = [[hipcc(), "-c", *HIPCC_FLAGS, *defs, src, "-o", obj] for src, defs, obj in units]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for r in ex.map(_run, cmds):
                if verbose and r.stderr:
                    print(r.stderr, file=sys.stderr)
        tmp_lib = out + ".tmp"
        _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *[u[2] for u in units],
              "-o", tmp_lib])
        os.replace(tmp_lib, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, verbose=a.v))
