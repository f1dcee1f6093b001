"""Build liblbsep.so (the C ABI of include/lbsep.h) for gfx950 with hipcc.

Usage: ``python -m paper_1603_08221_amd.build``. Cross-compiles without a GPU.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "lbsep.hip"), os.path.join(HERE, "csrc", "lbsep_adjoint.hip")]
OUT = os.path.join(HERE, "liblbsep.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # contract a*b+c only within one expression, so every kernel variant
    # rounds a given formula the same way (bitwise resume across variants)
    "-ffp-contract=on",
    # packed FP32 instructions stay off (the compiler would otherwise form them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source into liblbsep.so (always recompiles); returns its path."""
    fd, tmp = tempfile.mkstemp(prefix=".liblbsep.", suffix=".so.tmp", dir=HERE)
    os.close(fd)
    cmd = [hipcc(), *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        os.unlink(tmp)
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose:
        sys.stdout.write(res.stdout + res.stderr)
    os.chmod(tmp, 0o755)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
