"""Build libtmop.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1807_09807_amd.build

Objects go to <repo>/_build/, the library to paper_1807_09807_amd/libtmop.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtmop.so")
ARCH = os.environ.get("TMOP_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU
# instructions (v_pk_*_f32).  No fast-math: IEEE FP64 with FMA contraction.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(ROOT, "include")]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]


def sources(src_dir: str = CSRC):
    return sorted(f for f in os.listdir(src_dir) if f.endswith((".hip", ".cpp")))


def _compile(src: str, out_dir: str = OUT_DIR, extra=(), src_dir: str = CSRC) -> str:
    obj = os.path.join(out_dir, src + ".o")
    path = os.path.join(src_dir, src)
    if src.endswith(".hip"):
        cmd = ["hipcc", *HIP_FLAGS, *extra, "-c", path, "-o", obj]
    else:
        cmd = ["hipcc", *HOST_FLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(jobs: int | None = None, verbose: bool = True, lib: str = LIB, out_dir: str = OUT_DIR,
          extra=(), src_dir: str = CSRC) -> str:
    """Compile every source of `src_dir` (hipcc, gfx950) and link `lib`.
    `extra` adds compiler flags (e.g. -D tuning macros) for variant builds."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources(src_dir)
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)), 16)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, out_dir, tuple(extra), src_dir), srcs))
    tmp = lib + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build()
