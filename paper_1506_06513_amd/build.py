"""Build libflusi.so (HIP, gfx950) in-tree with hipcc.

Each grid size is its own translation unit so the compile runs in parallel.
Usage: python -m paper_1506_06513_amd.build [--jobs J] [--sanitize]
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


# Host-code sanitizer build (CPU only): AddressSanitizer and UndefinedBehavior-
# Sanitizer instrument the host side of every unit (the ABI, ensembles, the
# serving loop, the launchers); device code is built as usual.  A reduced grid
# list keeps it quick.  The library expects the ASan runtime preloaded
# (asan_runtime() gives its path).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LIB = os.path.join(HERE, "libflusi_asan.so")
SAN_SIZES = (16, 32)
SAN_BOXES = ((48, 32),)


def asan_runtime() -> str:
    import glob
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hits = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise FileNotFoundError("clang ASan runtime not found under ROCm's LLVM")
    return hits[-1]


def sources_hash() -> str:
    """Hash of the HIP sources and the header (tags the sanitized build)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(os.path.dirname(HERE), "include", "flusi.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sanitized_current() -> bool:
    tag = SAN_LIB[:-3] + ".sha"
    return os.path.exists(SAN_LIB) and os.path.exists(tag) and open(tag).read().strip() == sources_hash()


def build_sanitized(jobs: int | None = None, out: str = SAN_LIB) -> str:
    import shutil
    jobs = jobs or min(16, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="flusi_san_") as tmp:
        src = os.path.join(tmp, "pkg", "csrc")
        shutil.copytree(CSRC, src)
        os.makedirs(os.path.join(tmp, "include"))
        shutil.copy(os.path.join(os.path.dirname(HERE), "include", "flusi.h"), os.path.join(tmp, "include"))
        with open(os.path.join(src, "sizes.def"), "w") as f:
            f.writelines([f"FLUSI_SIZE({n})\n" for n in SAN_SIZES] + [f"FLUSI_BOX({a}, {b})\n" for a, b in SAN_BOXES])
        units = [(os.path.join(src, "flusi.hip"), [], os.path.join(tmp, "flusi.o")),
                 (os.path.join(src, "server.hip"), [], os.path.join(tmp, "server.o"))]
        units += [(os.path.join(src, "inst.hip"), [f"-DFLUSI_N={n}"], os.path.join(tmp, f"i{n}.o")) for n in SAN_SIZES]
        units += [(os.path.join(src, "inst.hip"), [f"-DFLUSI_NX={a}", f"-DFLUSI_N={b}"], os.path.join(tmp, f"i{a}x{b}.o"))
                  for a, b in SAN_BOXES]
        cmds = [[hipcc(), "-c", *HIPCC_FLAGS, *SAN_FLAGS, *defs, u, "-o", obj] for u, defs, obj in units]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(_run, cmds))
        _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-shared-libasan", *SAN_FLAGS,
              *[u[2] for u in units], "-o", out + ".tmp"])
        os.replace(out + ".tmp", out)
    if out == SAN_LIB:
        with open(SAN_LIB[:-3] + ".sha", "w") as f:
            f.write(sources_hash() + "\n")
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--sanitize", action="store_true", help="host ASan/UBSan build (libflusi_asan.so)")
    a = ap.parse_args()
    print(build_sanitized(a.jobs) if a.sanitize else build(a.jobs, verbose=a.v))
