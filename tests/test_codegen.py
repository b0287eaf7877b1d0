"""Generated-code checks for the FP64 stencil that requests its layers
straight into LDS (`k_op_dma`).  Its correctness rests on explicit
`s_waitcnt vmcnt` counts: per step a wave issues its layer requests
(`global_load_lds_dwordx4`) and exactly two 16-byte stores, and nothing else
that counts on the memory counter.  A spill, a split store or an extra load
in the loop would make the counts too small, and the LDS reads would race
with the requests in flight; these tests compile op.hip for gfx950 (no GPU
needed) and check the loops of both kernel variants (edge and interior tiles)."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2009_02171_amd import build as B


@pytest.fixture(scope="module")
def dma_loops():
    src = os.path.join(B.SRC, "op.hip")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "op.s")
        cmd = [B.HIPCC, *B.FLAGS, "-x", "hip", "-S", "--offload-device-only", "-o", out, src]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        text = open(out).read()
    m = re.search(r"^(_ZN3csd8k_op_dma\w*):[^\n]*\n(.*?)s_endpgm", text, re.S | re.M)
    assert m, "k_op_dma not found in the generated code"
    body = m.group(2).splitlines()
    # split into basic blocks; the compiler annotates each block of a loop
    # with its loop header
    loops, whole = {}, []
    header = None
    for line in body:
        lab = re.match(r"^(\.LBB\w+):|^; %bb\.\d+:", line)
        if lab:
            h = re.search(r"Header=(BB\w+)", line)
            if "Inner Loop Header" in line:
                header = lab.group(1)[2:]  # ".LBB3_7" -> "BB3_7", as in the annotations
            elif h:
                header = h.group(1)
            else:
                header = None
            continue
        ins = line.strip()
        if not ins or ins.startswith(";") or ins.startswith("."):
            continue
        whole.append(ins)
        if header:
            loops.setdefault(header, []).append(ins)
    return whole, loops


def _memory_ops(lines):
    return [ln.split()[0] for ln in lines if re.match(r"(global|scratch|buffer|flat)_", ln)]


def test_no_spills_or_flat_accesses(dma_loops):
    whole, _ = dma_loops
    ops = _memory_ops(whole)
    assert not [o for o in ops if not o.startswith("global_")], "scratch/buffer/flat access in k_op_dma"


def test_loop_memory_operations_are_the_counted_ones(dma_loops):
    _, loops = dma_loops
    assert len(loops) == 2, f"expected the edge and the interior loop, found {sorted(loops)}"
    for h, lines in loops.items():
        ops = _memory_ops(lines)
        # six unrolled steps: four requests (two in waves without extra
        # records, on a separate branch) and two 16-byte stores each
        assert set(ops) == {"global_load_lds_dwordx4", "global_store_dwordx4"}, (h, sorted(set(ops)))
        assert ops.count("global_store_dwordx4") == 12, (h, ops.count("global_store_dwordx4"))
        assert ops.count("global_load_lds_dwordx4") == 24, (h, ops.count("global_load_lds_dwordx4"))


def test_loop_waits_are_the_explicit_ones(dma_loops):
    """Only the per-step waits: 3P + 2M younger operations (P = 4 or 2
    requests per layer, M = 0..4); no compiler wait drains the pipeline."""
    _, loops = dma_loops
    allowed = {3 * p + 2 * m for p in (2, 4) for m in range(5)}
    for h, lines in loops.items():
        counts = [int(c) for ln in lines for c in re.findall(r"vmcnt\((\d+)\)", ln)]
        assert counts, h
        assert set(counts) <= allowed, (h, sorted(set(counts)))
        assert 0 not in counts, h
