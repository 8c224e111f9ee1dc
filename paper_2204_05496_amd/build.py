"""Build the HIP library liblrhe.so in-tree for gfx950 (hipcc cross-compiles; no GPU needed)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "liblrhe.so")
BUILD = os.path.join(HERE, "_build")

# (source, object, extra flags): the key-switch launchers build once per ring dimension
SOURCES = [("kernels.hip", "kernels.hip.o", []), ("host.cpp", "host.cpp.o", []), ("prof.cpp", "prof.cpp.o", []),
           ("plan.cpp", "plan.cpp.o", []), ("valu_rate.hip", "valu_rate.hip.o", []), ("wire.cpp", "wire.cpp.o", [])] + \
          [("ks_step.hip", f"ks_step.ln{ln}.o", [f"-DLRHE_KS_LOGN={ln}"]) for ln in range(10, 16)]
FLAGS = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
    # packed FP32 instructions stay off in every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fopenmp", "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(INCLUDE, "lrhe.h"))
    deps.append(os.path.abspath(__file__))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(entry, force: bool = False) -> str:
    src, oname, extra = entry
    obj = os.path.join(BUILD, oname)
    if not force and not _stale(obj, src):
        return obj
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {' '.join(extra)}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, force: bool = False) -> str:
    """Compile (objects whose sources or headers changed, or all with force) and link."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), max(2, os.cpu_count() or 2))) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-fopenmp", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, force="--force" in sys.argv)
    sys.exit(0)
