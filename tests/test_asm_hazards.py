"""Inline assembly next to the matrix cores (CPU: device assembly only).

The FP16 pair split of the matrix-core kernels is inline assembly
(`v_fma_mixlo/mixhi_f16` with operand selects that have no builtin).  The
compiler's hazard recognizer does not look inside inline assembly, so the
register allocator may hand an asm statement a VGPR that an MFMA issued just
before still has to write (a dead row of its result), and the MFMA's late
write would then clobber the asm result.  This test compiles the two
matrix-core sources to gfx950 assembly with the library's flags and checks,
in program order, that no inline-asm instruction writes or reads a VGPR in
the destination of an MFMA that is still in flight: one whose result no
later vector instruction has read (which makes the hardware wait for it)
within the following 64 vector instructions (at 4 or more cycles each, past
the longest MFMA latency).
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1808_10580_amd"))

WINDOW = 64


def _regs(tok):
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"-?v(\d+)", tok)
    if m:
        return {int(m.group(1))}
    return set()


def hazards(asm_text):
    """(function, instruction) pairs of inline-asm instructions that touch the
    destination of an MFMA still in flight, scanning each function in order."""
    found = []
    for body in re.split(r"\n(?=_Z\w+:)", asm_text):
        name = body.split(":", 1)[0]
        inflight = []  # [dst registers, vector instructions left in the window]
        in_asm = False
        for raw in body.split("\n"):
            line = raw.split(";;#")[0].strip() if not raw.strip().startswith(";;#") else raw.strip()
            if line.startswith(";;#ASMSTART"):
                in_asm = True
                continue
            if line.startswith(";;#ASMEND"):
                in_asm = False
                continue
            line = line.split(";")[0].strip()
            if not line or line.startswith(".") or line.endswith(":"):
                continue
            parts = line.replace(",", " ").split()
            op, ops = parts[0], parts[1:]
            regs = [_regs(t) for t in ops]
            if in_asm and op.startswith("v_"):
                touched = set().union(*regs) if regs else set()
                if any(touched & d for d, _ in inflight):
                    found.append((name, line))
            if op.startswith("v_mfma") and regs:
                inflight.append([regs[0], WINDOW])
            elif op.startswith("v_"):
                reads = set().union(*regs[1:]) if len(regs) > 1 else set()
                inflight = [[d, n - 1] for d, n in inflight if not (d & reads) and n > 1]
    return found


def _compile(src, extra):
    import build  # the library's own compile flags

    hipcc = build.HIPCC
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    out = subprocess.run([hipcc, *build.COMMON, *extra, "--cuda-device-only", "-S",
                          os.path.join(build.CSRC, src), "-o", "-"],
                         capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    return out.stdout


def test_checker_flags_a_planted_hazard():
    text = "\n".join([
        "_Zkernel:",
        "\tv_mfma_f32_32x32x16_f16 v[0:15], v[20:23], v[24:27], 0",
        "\t;;#ASMSTART",
        "\tv_fma_mixlo_f16 v3, v30, 1.0, -v31 op_sel_hi:[0,0,1]",
        "\t;;#ASMEND",
        "\tv_add_f32_e32 v40, v0, v41",
    ])
    assert len(hazards(text)) == 1
    # once a result of the MFMA has been read, the same asm is safe
    safe = text.replace("\t;;#ASMSTART", "\tv_add_f32_e32 v40, v0, v41\n\t;;#ASMSTART")
    assert hazards(safe) == []


@pytest.mark.parametrize("src", ["pm_mx.hip", "pm_hk.hip"])
def test_no_inline_asm_inside_an_mfma_in_flight(src):
    import build

    text = _compile(src, build.EXTRA.get(src, []))
    assert "v_mfma" in text and ";;#ASMSTART" in text
    bad = hazards(text)
    assert bad == [], bad[:5]
