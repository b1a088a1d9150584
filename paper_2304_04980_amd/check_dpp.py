"""Check the gfx950 assembly of the HIP sources for DPP read-after-write
hazards around the hand-written v_fmac_f32_dpp / v_fmac_f64_dpp
instructions.

A DPP instruction must not read a VGPR that a VALU instruction wrote fewer
than 2 instructions before it, nor follow a VALU write of EXEC by fewer than 5.
The compiler inserts the wait states for the DPP instructions it emits
itself but not for inline assembly, so every such FMA is checked here:
the previous instructions in program order, and every branch into a label
that falls inside that window.

    python -m paper_2304_04980_amd.check_dpp [source.hip ...]
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "--offload-device-only", "-S",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]

DPP_OPS = ("v_fmac_f32_dpp", "v_fmac_f64_dpp")
REG = re.compile(r"^v(\d+)$|^v\[(\d+):(\d+)\]$")


def regs(op: str) -> set[int]:
    m = REG.match(op.strip())
    if not m:
        return set()
    if m.group(1) is not None:
        return {int(m.group(1))}
    return set(range(int(m.group(2)), int(m.group(3)) + 1))


def parse(path: str):
    """Instruction list per function: (kind, text) with kind 'label' or 'ins'."""
    funcs, cur = {}, None
    for raw in open(path):
        line = raw.split(";")[0].rstrip()
        if not line.strip():
            continue
        s = line.strip()
        if s.endswith(":") and not s.startswith("."):
            cur = s[:-1]
            funcs[cur] = []
            continue
        if cur is None:
            continue
        if s.endswith(":"):
            funcs[cur].append(("label", s[:-1]))
        elif not s.startswith("."):
            funcs[cur].append(("ins", s))
    return funcs


def vgpr_writes(ins: str) -> set[int]:
    op = ins.split()[0]
    if not op.startswith("v_") or op.startswith(("v_cmp", "v_readlane", "v_readfirstlane")):
        return set()
    args = ins[len(op):].split(",")
    return regs(args[0]) if args else set()


def writes_exec(ins: str) -> bool:
    op = ins.split()[0]
    return op.startswith("v_cmpx") or (op.startswith("v_") and ins[len(op):].strip().startswith("exec"))


def check_func(name, body):
    problems = []
    labels = {b[1]: i for i, b in enumerate(body) if b[0] == "label"}
    branches = {}  # label -> indexes of branch instructions
    for i, (k, s) in enumerate(body):
        if k == "ins" and s.split()[0].startswith("s_cbranch") or (k == "ins" and s.startswith("s_branch")):
            tgt = s.split()[-1]
            branches.setdefault(tgt, []).append(i)

    def window(i, depth, seen=None):
        """Instruction sequences of length <= depth that can precede body[i]."""
        seen = seen or set()
        out = []
        j, got = i - 1, []
        while j >= 0 and len(got) < depth:
            k, s = body[j]
            if k == "label":
                for b in branches.get(s, []):
                    if (b, len(got)) in seen:
                        continue
                    seen.add((b, len(got)))
                    for tail in window(b + 1, depth - len(got), seen):
                        out.append(got + tail)
            else:
                got.append(s)
                if s.startswith("s_branch"):
                    return out
            j -= 1
        out.append(got)
        return out

    for i, (k, s) in enumerate(body):
        if k != "ins" or not s.startswith(DPP_OPS):
            continue
        src0 = regs(s.split(",")[1])
        for seq in window(i, 5):
            for d, prev in enumerate(seq):
                if d < 2 and vgpr_writes(prev) & src0:
                    problems.append(f"{name}: '{prev}' then '{s}'")
                if writes_exec(prev):
                    problems.append(f"{name}: exec write '{prev}' before '{s}'")
    return problems


def main(argv):
    srcs = argv or ["ops.hip", "batch.hip", "warm.hip"]
    bad, n = [], 0
    with tempfile.TemporaryDirectory() as tmp:
        for src in srcs:
            out = os.path.join(tmp, os.path.basename(src) + ".s")
            subprocess.run([HIPCC, *FLAGS, os.path.join(CSRC, src), "-o", out], check=True,
                           stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
            for name, body in parse(out).items():
                n += sum(1 for k, s in body if k == "ins" and s.startswith(DPP_OPS))
                bad += check_func(name, body)
    for b in bad[:20]:
        print(b)
    print(f"{n} DPP FMAs checked, {len(bad)} hazards")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
