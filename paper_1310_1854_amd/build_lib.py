"""Compile libvoronoi_rt.so (HIP, gfx950) in place.

    python -m paper_1310_1854_amd.build_lib

Every HIP source is compiled with the host-side sanity of plain IEEE
arithmetic: no fast-math and no FMA contraction (the FP64 path reproduces
the plain definition's rounding), and no packed FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvoronoi_rt.so")
SOURCES = ["scan.hip", "sort.hip", "build.hip", "trace.hip", "serve.hip"]
ARCH = os.environ.get("VRT_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int = 4, out: str = LIB, defines=()) -> str:
    """Compile every source and link the shared library at ``out``;
    ``defines`` are extra -D options (tuning knobs of the kernels)."""
    objs = []
    tag = "" if out == LIB else "." + os.path.basename(out).replace(".so", "")
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, s.replace(".hip", tag + ".o"))
        cmd = ["hipcc", "-c"] + [f for f in FLAGS if f != "-shared"] + [f"-D{d}" for d in defines] + [src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    cmd = ["hipcc"] + FLAGS + objs + ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def _drain(procs):
    failed = []
    for name, p in procs:
        out, _ = p.communicate()
        # hipcc's host pass does not know the GPU feature flag: harmless
        text = "\n".join(ln for ln in out.decode(errors="replace").splitlines()
                         if "is not a recognized feature for this target" not in ln)
        if p.returncode != 0:
            failed.append((name, text))
        elif text.strip():
            sys.stderr.write(text)
    procs.clear()
    if failed:
        for name, text in failed:
            sys.stderr.write(f"--- {name}\n{text}\n")
        raise RuntimeError("HIP compilation failed: " + ", ".join(n for n, _ in failed))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
