"""Checks on the gfx950 assembly of the FP8 inference kernel, compiled here
from the tree's sources with the library's flags (CPU only).

The kernel's scaled K = 64 products (v_mfma_scale_f32_32x32x64_f8f6f4) must
not have their A, B or scale registers rewritten between the instruction's
issue and the first read of its result: such writes reached the product
corrupted on the GPU (NaN outputs in some lanes).  The source keeps the
operands allocated until the sums are read; this test holds the compiler's
output to that, and to a kernel without scratch spills.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2108_05263_amd import build as B

KERNEL = "k_mlp_infer_fp8"

pytestmark = pytest.mark.skipif(not (os.path.exists(B.hipcc()) or shutil.which("hipcc")), reason="hipcc not found")


def _assembly(tmp_path, src):
    out = tmp_path / "gi_mlp.s"
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([B.hipcc()] + flags + ["--cuda-device-only", "-S", "-o", str(out), src], check=True,
                   capture_output=True)
    return out.read_text()


def _kernel_body(asm, name):
    m = re.search(r"^(_Z\S*" + name + r"\S*):", asm, re.M)
    assert m, f"{name} not found in the assembly"
    sym = m.group(1)
    start = m.end()
    end = asm.index("s_endpgm", start)
    return sym, [ln.strip() for ln in asm[start:end].splitlines()]


def _vregs(tok):
    tok = tok.strip()
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


_NO_VDST = ("ds_write", "global_store", "buffer_store", "scratch_store", "flat_store", "s_", "v_cmp", "v_readfirstlane",
            "v_readlane")


def _scaled_mfma_war(lines):
    """(mfma line, offending line) pairs: a vector register that a scaled
    product reads (A, B, scales, or an accumulator input other than its
    output) is written by a non-MFMA instruction before the product has
    completed.  Products complete in issue order, so the window closes at the
    first non-MFMA read of this or any later product's result; a later
    product may take the registers as its own output (written when it
    completes, after this one)."""
    found = []
    for i, ln in enumerate(lines):
        if not ln.startswith("v_mfma_scale"):
            continue
        ops = [o.strip() for o in ln.split(None, 1)[1].split(",")]
        pending = set(_vregs(ops[0]))
        src = set()
        for o in ops[1:]:
            src |= _vregs(o.split()[0])
        src -= _vregs(ops[0])   # accumulating in place: the input is the output
        for ln2 in lines[i + 1:i + 400]:
            if not ln2 or ln2.startswith((";", ".")):
                continue
            parts = ln2.split(None, 1)
            if len(parts) < 2:
                continue
            mnem, rest = parts
            ops2 = [o.strip() for o in rest.split(",")]
            if mnem.startswith("v_mfma"):
                pending |= _vregs(ops2[0])
                continue
            stores = mnem.startswith(_NO_VDST)
            reads = set()
            for o in (ops2 if stores else ops2[1:]):
                reads |= _vregs(o.split()[0])
            if reads & pending:
                break
            writes = set() if stores else _vregs(ops2[0])
            if writes & src:
                found.append((ln, ln2))
    return found


def test_scaled_mfma_operands_survive_until_results_are_read(tmp_path):
    asm = _assembly(tmp_path, os.path.join(B.CSRC, "gi_mlp.hip"))
    sym, body = _kernel_body(asm, KERNEL)
    n_mfma = sum(1 for ln in body if ln.startswith("v_mfma_scale_f32_32x32x64_f8f6f4"))
    assert n_mfma >= 11, n_mfma     # 11 products per 32-sample tile
    bad = _scaled_mfma_war(body)
    assert not bad, "\n".join(f"{a}  <-  {b}" for a, b in bad[:10])
    m = re.search(re.escape(sym) + r"\.private_seg_size, (\d+)", asm)
    assert m and int(m.group(1)) == 0, "the FP8 inference kernel spills to scratch"


def test_the_check_finds_an_early_operand_write():
    """The scan itself: a product whose B operand is overwritten right after
    issue is reported; the same write after the result's first read is not."""
    issue = "v_mfma_scale_f32_32x32x64_f8f6f4 v[0:15], v[16:23], v[24:31], v[0:15], v40, v41 op_sel_hi:[0,0,0]"
    early = [issue, "v_mov_b32_e32 v24, 0", "s_nop 7", "v_med3_f32 v50, v0, 0, v60"]
    late = [issue, "s_nop 15", "v_med3_f32 v50, v0, 0, v60", "v_mov_b32_e32 v24, 0"]
    scale = [issue, "v_mov_b32_e32 v41, 5", "v_add_f32_e32 v51, v2, v3"]
    # accumulator input v[64:79] reused as a later product's output: fine;
    # written by a VALU before either result is read: reported
    acc_in = "v_mfma_scale_f32_32x32x64_f8f6f4 v[0:15], v[16:23], v[24:31], v[64:79], v40, v41 op_sel_hi:[0,0,0]"
    reuse = [acc_in, "v_mfma_scale_f32_32x32x64_f8f6f4 v[64:79], v[16:23], v[32:39], v[64:79], v40, v41",
             "s_nop 15", "v_med3_f32 v50, v64, 0, v60", "v_mov_b32_e32 v70, 0"]
    clobber = [acc_in, "v_mov_b32_e32 v70, 0", "s_nop 15", "v_med3_f32 v50, v0, 0, v60"]
    assert _scaled_mfma_war(early) == [(issue, "v_mov_b32_e32 v24, 0")]
    assert _scaled_mfma_war(late) == []
    assert _scaled_mfma_war(scale) == [(issue, "v_mov_b32_e32 v41, 5")]
    assert _scaled_mfma_war(reuse) == []
    assert _scaled_mfma_war(clobber) == [(acc_in, "v_mov_b32_e32 v70, 0")]
