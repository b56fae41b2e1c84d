"""Build step for libiod.so (gfx950) -- compiled in-tree with hipcc.

Flags that matter for results:
  -ffp-contract=off   the compiler fuses no multiply-add; every fma is
                      explicit in the source, so the FP64 evaluation order
                      is the one written there.
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions are generated.

A flag that matters for speed only, per source file:
  -mllvm -amdgpu-sched-strategy=max-ilp (FP64 swarm kernels)
                      the instruction scheduler favours latency hiding over
                      register count. The single large swarm runs one wave
                      per SIMD, so nothing else hides the dependency
                      latency; the batched FP64 kernel keeps its 2 waves per
                      SIMD. Not used for the FP32 kernels, whose occupancy
                      (5 waves per SIMD) it would cut to 3.
Each file is compiled on its own (none references another's device code)
and the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libiod.so")
MAX_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
# (source, extra flags)
UNITS = [("iod_kernels.hip", MAX_ILP), ("iod_mixed.hip", []), ("iod_sens.hip", []),
         ("iod_api.hip", [])]
SOURCES = [os.path.join(CSRC, f) for f, _ in UNITS]

ARCH = ["--offload-arch=gfx950"]
LIBS = ["-lrocprofiler-sdk-roctx"]   # phase ranges for marker-recording tools
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run_all(cmds):
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
             for c in cmds]
    out, failed = [], []
    for c, p in procs:
        text = p.communicate()[0]
        out.append(text)
        if p.returncode != 0:
            failed.append(" ".join(c) + "\n" + text)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    return "".join(out)


def build(verbose: bool = False) -> str:
    tmpdir = tempfile.mkdtemp(prefix="iod_build_")
    try:
        objs = [os.path.join(tmpdir, f.replace(".hip", ".o")) for f, _ in UNITS]
        text = _run_all([[hipcc(), *ARCH, *FLAGS, *extra, "-c", "-o", o, os.path.join(CSRC, f)]
                         for (f, extra), o in zip(UNITS, objs)])
        tmp = LIB + ".tmp"
        text += _run_all([[hipcc(), *ARCH, "-shared", "-fPIC", "-o", tmp, *objs, *LIBS]])
        if verbose:
            print(text)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


def device_asm(out_path: str, source: str = "iod_kernels.hip") -> str:
    """Write the gfx950 assembly of one source file's kernels (for inspection)."""
    extra = dict(UNITS)[source]
    cmd = [hipcc(), *ARCH, *FLAGS, *extra, "--offload-device-only", "-S", "-o", out_path,
           os.path.join(CSRC, source)]
    subprocess.run(cmd, check=True)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
