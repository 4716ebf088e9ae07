"""Build libeloc.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_2408_07625_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libeloc.so"
SOURCES = [CSRC / "kernels.hip", CSRC / "pairs.hip", CSRC / "batch.hip", CSRC / "misses.hip", CSRC / "sr.hip", CSRC / "sampler.hip",
           CSRC / "api.cpp",
           CSRC / "batch.cpp"]
HEADERS = [CSRC / "internal.h", CSRC / "device.h", CSRC / "trie.h", CSRC / "ham.h", CSRC / "host.h",
           ROOT / "include" / "eloc.h"]

# Packed-FP32 instructions are disabled for all HIP code (the compiler would
# otherwise pair scalar FP32 adds/multiplies into v_pk_* forms).  Floating-
# point contraction is off: the error-free transforms of the compensated FP32
# path need every product rounded on its own (fused multiply-adds are written
# out explicitly where they are wanted).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, incremental: bool = False) -> Path:
    """Compile every source to an object file (in parallel), then link.
    incremental: keep object files newer than their source and every header."""
    obj_dir = PKG / "_build"
    obj_dir.mkdir(exist_ok=True)
    inc = [f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs = []
    newest_header = max(h.stat().st_mtime for h in HEADERS)
    for src in SOURCES:
        obj = obj_dir / (src.name + ".o")
        if incremental and obj.exists() and obj.stat().st_mtime > max(src.stat().st_mtime, newest_header):
            procs.append((src, obj, None))
            continue
        cmd = [hipcc(), *compile_flags, *inc, "-c", str(src), "-o", str(obj)]
        procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                  text=True)))
    logs, failed = [], False
    for src, obj, p in procs:
        if p is None:
            continue
        out, _ = p.communicate()
        logs.append(out)
        failed = failed or p.returncode != 0
    if failed:
        sys.stderr.write("\n".join(logs))
        raise RuntimeError("hipcc failed")
    tmp = LIB.with_name(LIB.name + ".tmp")
    res = subprocess.run([hipcc(), *FLAGS, *[str(o) for _, o, _ in procs], "-o", str(tmp)], capture_output=True,
                         text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    if verbose:
        noise = ("packed-fp32-ops", "is not a recognized feature")
        for line in ("\n".join(logs) + res.stdout + res.stderr).splitlines():
            if line.strip() and not any(n in line for n in noise):
                print(line)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not LIB.exists():
        return True
    t = LIB.stat().st_mtime
    return any(p.stat().st_mtime > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
