"""Build libkf.so (HIP kernels + C interface) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkf.so")
SOURCES = ["kf_api.hip", "kf_kernels.hip", "kf_adjoint.hip", "kf_search.hip", "kf_backward.hip", "kf_dedup.hip", "kf_final.hip",
           "kf_plane.hip"]
ARCH = os.environ.get("KF_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# roctx ranges name each interface call on a profiler's timeline
LIBS = ["-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # the compiler's default floating-point contraction, unless
         # KF_FP_CONTRACT names another mode (on, fast, off)
         "-Wno-unused-command-line-argument"]
if os.environ.get("KF_FP_CONTRACT"):
    FLAGS.append("-ffp-contract=" + os.environ["KF_FP_CONTRACT"])


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def compile_commands(build_dir: str, out: str) -> tuple[list[list[str]], list[str]]:
    """One hipcc -c per source (run in parallel), then the link of libkf.so."""
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc()] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs + LIBS
    return cmds, link


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="kf_build_") as bd:
        cmds, link = compile_commands(bd, tmp)
        if verbose:
            for c in cmds + [link]:
                print(" ".join(c), flush=True)
        procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True) for c in cmds]
        outs = [(p.communicate()[0], p.returncode) for p in procs]
        for out, rc in outs:
            if rc != 0:
                sys.stderr.write(out)
        if any(rc != 0 for _, rc in outs):
            raise RuntimeError("hipcc failed building libkf.so")
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libkf.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
