"""Build libqpx.so (HIP kernels + C-ABI) for gfx950 with hipcc, in-tree.

Each kernel configuration is its own translation unit so the objects
compile in parallel; objects go to csrc/_build/ (not committed)."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libqpx.so")
# profiling builds: extra compiler flags and an output path of their own
EXTRA = os.environ.get("QPX_EXTRA_FLAGS", "").split()
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 VALU ops are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-pthread",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _newest_dependency() -> float:
    """Newest modification time of the headers every unit includes."""
    deps = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.h"))
    deps.append(os.path.join(HERE, "..", "include", "qpx.h"))
    return max(os.path.getmtime(d) for d in deps)


def _compile(src: str, extra=(), incremental: bool = False) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(src), _newest_dependency()):
        return obj
    cmd = [HIPCC, *FLAGS, *EXTRA, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None, out: str | None = None,
          objdir: str | None = None, incremental: bool = False) -> str:
    """Compile every unit (or, with incremental, only units older than their
    sources) and link libqpx.so."""
    global OBJ
    if objdir:
        OBJ = objdir
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental=incremental), srcs))
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libqpx.so")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
