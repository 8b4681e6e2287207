"""Build kf_host_check: the per-track host-device code of the HIP path
compiled for the host only, under the address and undefined-behaviour
sanitizers (hipcc, no GPU code is generated).

    python tests/hostcheck/build.py [output]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2312_11728_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SOURCE = os.path.join(HERE, "kf_host_check.cpp")


def hipcc() -> str | None:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def command(out: str) -> list[str]:
    # host-only compilation; each sanitizer flag is scoped to the host pass
    return [hipcc(), "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Wno-unused-command-line-argument",
            "-I", INCLUDE, "-I", CSRC, SOURCE, "-o", out]


def build(out: str) -> str:
    if hipcc() is None:
        raise RuntimeError("hipcc not found")
    r = subprocess.run(command(out), capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building kf_host_check")
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "kf_host_check")))
