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
import functools
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


@functools.lru_cache(maxsize=None)
def _compile_cached(src, extra):
    return _compile(src, list(extra))


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

    text = _compile_cached(src, tuple(build.EXTRA.get(src, [])))
    assert "v_mfma" in text and ";;#ASMSTART" in text
    bad = hazards(text)
    assert bad == [], bad[:5]


# ---------------------------------------------------------------------------
# The cooperative disk tail runs one walker per wave: lane 0 takes the next
# walker index from the pool and a shuffle gives it to the other lanes, and
# every loop of the kernel is left by the whole wave together (the walker's
# state, and so each exit condition, is the same in every lane).  A loop that
# the compiler lets lanes leave one by one is closed by an exec-mask update
# `s_andn2_b64 exec, exec, ...`; once, a lane-0 branch that ended the walker
# loop was merged with the next walker's lane-0 fetch in that way, so lanes
# 1-63 re-entered the shuffle without lane 0 and walked a stale walker.
# ---------------------------------------------------------------------------
def functions(asm_text):
    """(name, body) of each function in a device assembly listing."""
    out = []
    for body in re.split(r"\n(?=_Z\w+:)", asm_text):
        name = body.split(":", 1)[0].strip()
        if name.startswith("_Z"):
            out.append((name, body.split(".Lfunc_end", 1)[0]))
    return out


def lane_by_lane_loop_exits(body):
    return [l.strip() for l in body.split("\n") if l.strip().startswith("s_andn2_b64 exec, exec")]


def test_loop_exit_check_flags_a_lane_by_lane_exit():
    text = "\n".join([
        "_Zkernel:",
        ".LBB0_1:",
        "\ts_or_b64 s[48:49], s[80:81], s[48:49]",
        "\ts_andn2_b64 exec, exec, s[48:49]",
        "\ts_cbranch_execnz .LBB0_1",
        ".Lfunc_end0:",
    ])
    (name, body), = functions(text)
    assert name == "_Zkernel" and len(lane_by_lane_loop_exits(body)) == 1
    assert lane_by_lane_loop_exits(body.replace("s_andn2_b64 exec, exec", "s_andn2_b64 vcc, exec")) == []


def test_disk_tail_loops_are_left_by_the_whole_wave():
    import build

    text = _compile_cached("pm_mx.hip", tuple(build.EXTRA.get("pm_mx.hip", [])))
    tails = [(n, b) for n, b in functions(text) if "k_dirichlet_tail" in n]
    assert len(tails) == 8  # K = 1..4, zero/constant/linear and general sources
    for name, body in tails:
        assert lane_by_lane_loop_exits(body) == [], name
