"""Host-side sanitizer builds for the CPU test tier: a copy of libiod whose
host code (argument checks, layouts, the C ABI) is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer, and a copy of the oracle
built the same way. Device code is compiled as usual: the sanitizers apply to
host code only. Loaded in a child process with the sanitizer runtime
preloaded (python itself is not instrumented)."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import tempfile

HIP_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split() + \
    ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def clang_asan_runtime() -> str | None:
    """The ASan runtime of the compiler that builds libiod's host code."""
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def gcc_asan_runtime() -> str | None:
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def build_libiod(out_path: str) -> str:
    from paper_2207_13175_amd import build as B
    tmp = tempfile.mkdtemp(prefix="iod_san_")
    try:
        objs, procs = [], []
        flags = [x for x in B.FLAGS if x != "-O3"] + ["-O1", "-g"]
        for f, _ in B.UNITS:
            o = os.path.join(tmp, f.replace(".hip", ".o"))
            procs.append(subprocess.Popen([B.hipcc(), *B.ARCH, *flags, *HIP_SAN, "-c", "-o", o,
                                           os.path.join(B.CSRC, f)],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
            objs.append(o)
        for pr in procs:
            out = pr.communicate()[0]
            if pr.returncode != 0:
                raise RuntimeError(out.decode(errors="replace"))
        subprocess.run([B.hipcc(), *B.ARCH, "-shared", "-fPIC", *HIP_SAN, "-shared-libsan",
                        "-o", out_path, *objs, *B.LIBS], check=True, capture_output=True)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out_path


def build_oracle(out_path: str) -> str:
    import oracle
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", *GCC_SAN, "-o", out_path, oracle._SRC, "-lm"], check=True)
    return out_path
