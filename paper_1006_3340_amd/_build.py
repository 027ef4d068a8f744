"""Compile the HIP sources of the package into liblll.so (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblll.so")
SOURCES = ["abi.hip", "precompute.hip", "paths.hip", "batched.hip", "adjoint.hip",
           "mlp_train.hip", "mlp_path.hip", "mlp_host.hip", "picard_mp.hip",
           "fma_probe.hip", "exact.hip", "noalloc.hip"] + sorted(
    f for f in os.listdir(CSRC) if f.startswith(("bucket_", "adjoint_b", "batched_b")) and f.endswith(".hip"))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]


# The path kernels keep their whole state in registers; hoisting the FP64
# constants of the increment's log/sincos out of the step loop would pin ~40
# VGPRs for the kernel's lifetime, so machine-level loop-invariant code motion
# is off for those translation units (the uniform table reads stay scalar).
PATH_FLAGS = ["-mllvm", "-disable-machine-licm"]


def _headers_mtime() -> float:
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    heads += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(h) for h in heads + [os.path.abspath(__file__)])


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not force and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _headers_mtime():
            return obj
    extra = PATH_FLAGS if src.startswith(("bucket_", "batched", "adjoint", "mlp_")) else []
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force) or only those older than their inputs."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda f: _compile(f, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True, force="--changed" not in sys.argv)
