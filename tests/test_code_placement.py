"""Where the FP32 iteration kernel's hot RK4 loop lands in its code object.

The absolute-state instances of k_mixed_iter run the uneven batch's
iteration in 15.8-16.5 ms when the loop starts at 8 or 16 mod 32 bytes and
in 17.8-19.0 ms at the other six offsets, with the same instructions. Their
entry paddings (iter_pad in iod_mixed.hip) are chosen to land at 8 mod 32.
An edit to that file or to the device code it includes moves the loops;
this test then names each instance that left the fast offsets, so that its
padding can be retuned. It compiles the file's device code (hipcc for
gfx950, no GPU needed) and reads the disassembly of that compiled code."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2207_13175_amd import build as B

LLVM = "/opt/rocm/llvm/bin"
FAST = {8, 16}


def _tools():
    paths = [B.hipcc(), os.path.join(LLVM, "clang-offload-bundler"), os.path.join(LLVM, "llvm-objdump")]
    if not all(shutil.which(p) or os.path.exists(p) for p in paths):
        pytest.skip("ROCm compiler tools not found")
    return paths


def _hot_loops(dis):
    """{kernel: start address} of each kernel's innermost backward-branch
    loop that holds at least 8 v_rsq (one RK4 step, two per stage)."""
    funcs, base, cur = {}, {}, None
    for line in dis.splitlines():
        m = re.match(r"^([0-9a-f]+) <(\S+)>:", line)
        if m:
            cur = m.group(2)
            funcs[cur], base[cur] = [], int(m.group(1), 16)
            continue
        m = re.match(r"^\s+(\S+)\s*(.*?)\s*//\s*([0-9A-F]+):", line)
        if m and cur:
            funcs[cur].append((int(m.group(3), 16), m.group(1), line))
    out = {}
    for f, ins in funcs.items():
        best = None
        for a, op, line in ins:
            if not (op.startswith("s_cbranch") or op == "s_branch"):
                continue
            t = re.search(r"<\S+\+0x([0-9a-f]+)>", line)
            if not t:
                continue
            tgt = base[f] + int(t.group(1), 16)
            if tgt < a and sum(1 for x in ins if tgt <= x[0] <= a and x[1].startswith("v_rsq")) >= 8:
                if best is None or a - tgt < best[1] - best[0]:
                    best = (tgt, a)
        if best:
            out[f] = best[0]
    return out


def test_absolute_iteration_loops_start_at_fast_offsets(tmp_path):
    hipcc, bundler, objdump = _tools()
    obj, co = tmp_path / "mixed.o", tmp_path / "mixed.co"
    subprocess.run([hipcc, *B.ARCH, *B.FLAGS, *dict(B.UNITS)["iod_mixed.hip"], "--offload-device-only",
                    "-c", "-o", str(obj), os.path.join(B.CSRC, "iod_mixed.hip")],
                   check=True, capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o", f"--input={obj}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                   check=True, capture_output=True)
    dis = subprocess.run([objdump, "-d", "--no-show-raw-insn", str(co)], check=True,
                         capture_output=True, text=True).stdout
    loops = _hot_loops(dis)
    absolute = {f: a for f, a in loops.items() if re.search(r"k_mixed_iterILi\d+ELb0E", f)}
    assert len(absolute) == 3, sorted(loops)
    off = {re.search(r"ILi(\d+)E", f).group(1): a % 32 for f, a in absolute.items()}
    bad = {bs: o for bs, o in off.items() if o not in FAST}
    assert not bad, f"k_mixed_iter<BS, false> hot loop at {bad} mod 32 (fast: {sorted(FAST)})"
