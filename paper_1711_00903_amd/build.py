"""Build ``libfem.so`` (the HIP kernels and the C ABI of ``include/fem.h``) for gfx950.

Each source is compiled separately with ``hipcc`` (in parallel), then linked
into ``paper_1711_00903_amd/libfem.so``.  Object files go to ``_build/``.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfem.so")

PRECS = ["f64", "f32", "bf16", "f16", "bf16g", "f16g", "f32g64", "bf16g64", "f16g64"]
SOURCES = ["fem_api.cpp", "batch.cpp", "basis.cpp", "geometry.hip", "cg.hip", "assembled.hip", "bp35v.hip",
           "bp30v.hip",
           "cgop_f64.hip", "cgop_f32g64.hip", "cgop_bf16g64.hip", "cgop_f16g64.hip"] + [
    f"{op}_{p}.hip" for op in ("bp35", "bp10", "bp30") for p in PRECS]

ARCH = os.environ.get("FEM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def source_hash() -> str:
    """Hash of the library's sources (csrc/ and include/fem.h): names and
    contents, in name order.  The build compiles it into the library, where
    ``fem_build_id()`` returns it, so a library built from other sources than
    the checkout's is detected."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp", ".h")))
    for name, path in [(f, os.path.join(CSRC, f)) for f in files] + [("fem.h", os.path.join(INCLUDE, "fem.h"))]:
        h.update(name.encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(INCLUDE, "fem.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, verbose: bool, incremental: bool = False, build_id: str = "") -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
    stamp = obj + ".id"
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(path), _newest_header()) and \
            (not build_id or (os.path.exists(stamp) and open(stamp).read() == build_id)):
        return obj
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj]
    if build_id:
        cmd.append(f'-DFEM_BUILD_ID="{build_id}"')
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if build_id:
        with open(stamp, "w") as fh:
            fh.write(build_id)
    return obj


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source for gfx950 and link ``libfem.so``; returns its path.
    With ``incremental``, objects newer than their source and every header are kept."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    bid = source_hash()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        # the ABI unit carries the source hash (fem_build_id)
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental, bid if s == "fem_api.cpp" else ""),
                           SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
