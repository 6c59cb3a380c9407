"""Generated-code check of the MFMA kernels (CPU: hipcc cross-compiles gfx950).

A matrix instruction writes its accumulator some cycles after it issues; a
v_accvgpr_read of that accumulator must come later than that, and the
compiler pads such reads with s_nop to at least ten wait states after an FP32
or FP64 16x16x4 MFMA in straight-line code.  A kernel whose control flow gives
the compiler a join of several paths can end up with a shorter path: the
theta kernel with three K-chunks in flight had one of three wait states in
its complex64 build, and its results were wrong on the GPU.  This test
compiles the kernels that use MFMA with the library's own flags and walks
every path backwards from each accumulator read (through fall-through and
branch edges) to the last MFMA that wrote the register.  On gfx950 an MFMA
can also write ordinary VGPRs; a VALU instruction (or another MFMA's A or B
operand) reading such a result needs eleven wait states after an FP64
16x16x4 MFMA, a memory instruction eighteen, and the second check walks every
VGPR read the same way.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_1703_00387_amd import build as B

MFMA_SOURCES = ["theta.hip", "gemm.hip", "heff.hip", "svd.hip", "warm.hip"]
MIN_WAIT = 10
SEARCH = 30


def _agprs(tok):
    m = re.match(r"a\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"a(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _items(body):
    items = []
    for line in body.splitlines():
        line = line.split(";")[0].strip()
        if not line or (line.startswith(".") and not line.endswith(":")):
            continue
        items.append(("label", line[:-1]) if line.endswith(":") else ("ins", line))
    return items


def short_reads(body):
    """(wait states, read) for every accumulator read closer than MIN_WAIT to
    the MFMA that wrote it, along some path of the function body."""
    items = _items(body)
    branches = {}
    for i, (k, t) in enumerate(items):
        if k == "ins" and (t.startswith("s_cbranch") or t.startswith("s_branch")):
            branches.setdefault(t.split()[-1], []).append(i)

    def back(i, reg, dist, seen):
        best = None
        j = i - 1
        while j >= 0 and dist < SEARCH:
            k, t = items[j]
            if k == "label":
                for b in branches.get(t, []):
                    if (b, reg) not in seen:
                        seen.add((b, reg))
                        r = back(b + 1, reg, dist, seen)
                        if r is not None and (best is None or r < best):
                            best = r
                j -= 1
                continue
            if t.startswith("s_branch") or t.startswith("s_endpgm"):
                return best
            if t.startswith("v_mfma") and reg in _agprs(t.split()[1].strip(",")):
                return dist if best is None else min(best, dist)
            dist += int(t.split()[1]) + 1 if t.startswith("s_nop") else 1
            j -= 1
        return best

    out = []
    for i, (k, t) in enumerate(items):
        if k == "ins" and t.startswith("v_accvgpr_read"):
            reg = min(_agprs(t.split()[2].strip(",")))
            d = back(i, reg, 0, set())
            if d is not None and d < MIN_WAIT:
                out.append((d, t))
    return out


def test_analysis_finds_a_short_path():
    """The walk sees a read three wait states after the MFMA across a taken
    branch, and accepts one padded to ten."""
    bad = """f:
\tv_mfma_f32_16x16x4_f32 a[0:3], v1, v2, a[0:3]
\ts_and_saveexec_b64 s[2:3], s[4:5]
\ts_cbranch_execz .LBB0_2
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
.LBB0_2:
\ts_or_b64 exec, exec, s[2:3]
\tv_accvgpr_read_b32 v9, a2
\ts_endpgm
"""
    assert [d for d, _ in short_reads(bad)] == [3]
    good = bad.replace("\ts_or_b64 exec, exec, s[2:3]\n", "\ts_or_b64 exec, exec, s[2:3]\n\ts_nop 6\n")
    assert short_reads(good) == []


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


VGPR_WAIT = {"valu": 11, "mfma_ab": 11, "mem": 18}
_MEM_READS_ALL = ("ds_write", "ds_store", "global_store", "buffer_store", "flat_store", "global_atomic",
                  "ds_add", "ds_bpermute", "ds_permute")
_MEM_LOADS = ("global_load", "buffer_load", "ds_read", "ds_load", "flat_load", "scratch_load")


def _vgpr_reads(t):
    parts = t.split(None, 1)
    op = parts[0]
    o = [x.strip().split()[0] for x in parts[1].split(",")] if len(parts) > 1 else []
    if op.startswith("v_mfma"):
        src, kind = o[1:3], "mfma_ab"
    elif op.startswith(_MEM_READS_ALL):
        src, kind = o, "mem"
    elif op.startswith(_MEM_LOADS):
        src, kind = o[1:], "mem"
    elif op.startswith("v_"):
        src, kind = (o if op.startswith("v_cmp") else o[1:]), "valu"
    else:
        return set(), None
    regs = set()
    for x in src:
        regs |= _vregs(x)
    return regs, kind


def short_vgpr_reads(body):
    """(wait states, kind, instruction) for every read of an MFMA's VGPR
    result closer than VGPR_WAIT along some path of the function body."""
    items = _items(body)
    branches = {}
    for i, (k, t) in enumerate(items):
        if k == "ins" and (t.startswith("s_cbranch") or t.startswith("s_branch")):
            branches.setdefault(t.split()[-1], []).append(i)

    def back(i, regs, dist, seen):
        best = None
        j = i - 1
        while j >= 0 and dist < SEARCH:
            k, t = items[j]
            if k == "label":
                for b in branches.get(t, []):
                    if (b, i) not in seen:
                        seen.add((b, i))
                        r = back(b + 1, regs, dist, seen)
                        if r is not None and (best is None or r < best):
                            best = r
                j -= 1
                continue
            if t.startswith("s_branch") or t.startswith("s_endpgm"):
                return best
            if t.startswith("v_mfma") and _vregs(t.split()[1].strip(",")) & regs:
                return dist if best is None else min(best, dist)
            dist += int(t.split()[1]) + 1 if t.startswith("s_nop") else 1
            j -= 1
        return best

    out = []
    for i, (k, t) in enumerate(items):
        if k != "ins":
            continue
        regs, kind = _vgpr_reads(t)
        if kind is None or not regs:
            continue
        d = back(i, regs, 0, set())
        if d is not None and d < VGPR_WAIT[kind]:
            out.append((d, kind, t))
    return out


def test_vgpr_analysis_finds_a_short_path():
    """A VALU read of an MFMA's VGPR result four wait states later across a
    taken branch is found; padded to eleven it is accepted."""
    bad = """f:
\tv_mfma_f64_16x16x4_f64 v[10:17], v[2:3], v[4:5], v[10:17]
\ts_cbranch_execz .LBB0_2
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
\tv_add_f32_e32 v5, v6, v7
.LBB0_2:
\ts_or_b64 exec, exec, s[2:3]
\ts_nop 1
\tv_add_f64 v[20:21], v[12:13], v[30:31]
\ts_endpgm
"""
    assert [(d, k) for d, k, _ in short_vgpr_reads(bad)] == [(4, "valu")]
    good = bad.replace("\ts_nop 1\n", "\ts_nop 8\n")
    assert short_vgpr_reads(good) == []


def _compile(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src)[:-4] + ".s")
    cmd = [B.hipcc(), *[f for f in B.FLAGS if f != "-fPIC"], "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
def test_no_accumulator_read_inside_mfma_latency(tmp_path):
    srcs = [os.path.join(B.CSRC, f) for f in MFMA_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        outs = list(ex.map(lambda s: _compile(s, str(tmp_path)), srcs))
    found, found_v, n_kernels, n_mfma = [], [], 0, 0
    for out in outs:
        text = open(out).read()
        for m in re.finditer(r"^(_Z\w+):.*?s_endpgm", text, re.M | re.S):
            n_kernels += 1
            n_mfma += m.group(0).count("v_mfma")
            found += [(os.path.basename(out), m.group(1), d, t) for d, t in short_reads(m.group(0))]
            found_v += [(os.path.basename(out), m.group(1), d, k, t) for d, k, t in short_vgpr_reads(m.group(0))]
    assert n_kernels > 20 and n_mfma > 1000, (n_kernels, n_mfma)
    assert not found, found[:5]
    assert not found_v, found_v[:5]
