"""Build libtxe.so (HIP kernels for gfx950 + the C-ABI host library) in-tree.

    python -m paper_2401_04189_amd.build [--verbose]

Every call recompiles.  The library is written next to this file.
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtxe.so")

SOURCES = ["txe_core_f32_5.hip", "txe_core_f32_4.hip", "txe_core_f32.hip", "txe_core_f64.hip",
           "txe_core_f64_45.hip", "txe_core_bf16.hip", "txe_back.hip", "txe_proj.hip", "txe_chunk.hip", "txe_pairbases.hip",
           "txe_ace.hip", "txe_ceiling.hip", "txe_scratch.hip", "txe_modes.hip", "txe_colloc.hip", "txe_hosvd.hip", "txe_api.cpp", "txe_setup.cpp", "txe_fe.cpp"]
ARCH = "gfx950"


def hipcc():
    p = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return p if os.path.exists(p) else "hipcc"


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed-FP32 instructions anywhere in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        f"-I{os.path.join(ROOT, 'include')}",
    ]


def _compile(src, extra, verbose):
    obj = os.path.join(HERE, "_build", src + ".o")
    cmd = [hipcc(), *flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    return obj, " ".join(shlex.quote(c) for c in cmd), out


def build(verbose=False, extra=(), jobs=None):
    """Compiles every source (in parallel, at most `jobs` at once) and links."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(lambda src: _compile(src, extra, verbose), SOURCES))
    objs = []
    for obj, cmd, out in res:
        if verbose:
            print(cmd, flush=True)
            if out:
                print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    v = "--verbose" in sys.argv
    extra = ["-Rpass-analysis=kernel-resource-usage"] if "--resource-usage" in sys.argv else []
    print(build(verbose=v or bool(extra), extra=extra))
