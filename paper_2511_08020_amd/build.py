"""Build libpolydg.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpolydg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_SOURCES = ["tables.cpp", "balance.cpp", "api.cpp"]
DEVICE_SOURCES = ["kernels.hip", "adjoint.hip", "batch.hip", "split.hip", "check.hip", "noalloc.hip", "motion.hip"]
OBJDIR = os.path.join(HERE, "_build")


def _filter(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link libpolydg.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs, objs = [], []
    for src in HOST_SOURCES + DEVICE_SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + compile_flags + ["-c"] + lang + [os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for cmd, p in jobs:
        out, _ = p.communicate()
        msgs = _filter(out)
        if p.returncode != 0:
            failed.append(f"hipcc failed ({p.returncode}):\n{' '.join(cmd)}\n{msgs}")
        elif verbose and msgs.strip():
            print(msgs, file=sys.stderr)
    if failed:
        raise RuntimeError("\n".join(failed))
    tmp = OUT + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed ({res.returncode}):\n{' '.join(cmd)}\n{_filter(res.stdout + res.stderr)}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
