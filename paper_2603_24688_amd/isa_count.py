"""VALU instructions per decode round of the binary32 pair passes, counted in
the gfx950 assembly of the library (the per-pair work that the benchmark's
VALU roofline uses).

    python -m paper_2603_24688_amd.isa_count

compiles the library's device code to assembly (hipcc -S, about a minute) and,
for k_pass_dm<float, 0> and k_pass_gas<float, 0, exact rates>, finds the loop
that evaluates one round of 64 pairs (lane = pair): the loop holding the
segmented scans over the round's lanes (the block with the most row_bcast:31
moves of the kernel).  It sums the vector-ALU
instructions of that loop's blocks at the loop's own depth: hit decode,
binary64 distance recheck, pair body and reductions, once per round.  Each
such wave instruction does one pair's share on every lane, so the count is
also the lane-instructions per pair.  The blocks of the per-pair minimum image
(a binary64 division and rounding per axis, marked by v_rndne_f64) run only
for sub-tiles that straddle a periodic boundary and are left out; the other
conditional blocks are included.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from collections import Counter

from . import build as _build

KERNELS = {
    "pass_dm": "_ZN3dmb9k_pass_dmIfLi0ELb0ELb0E",
    "pass_gas": "_ZN3dmb10k_pass_gasIfLi0ELb0ELi0ELb0E",
}


def assemble(out_s: str) -> None:
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [_build.hipcc(), *flags, "-I", os.path.join(_build.ROOT, "include"), "--cuda-device-only", "-S",
           "-o", out_s, os.path.join(_build.CSRC, "dmb_api.hip")]
    subprocess.run(cmd, check=True, capture_output=True)


def _blocks(body):
    out, i = [], 0
    while i < len(body):
        m = re.match(r"^\.(LBB\S+):(.*)", body[i])
        if not m:
            i += 1
            continue
        name, info, j = m.group(1), m.group(2), i + 1
        while j < len(body) and body[j].strip().startswith(";"):
            info += " " + body[j]
            j += 1
        ins = []
        while j < len(body) and not re.match(r"^\.LBB", body[j]):
            t = body[j].strip()
            if t and not t.startswith(";") and not t.startswith("."):
                ins.append(t)
            j += 1
        own = re.search(r"Loop Header: Depth=(\d)", info)
        h = re.search(r"Header=(\S+)\s+Depth=(\d)", info)
        if own:
            hdr, d = name, int(own.group(1))
        elif h:
            hdr, d = h.group(1), int(h.group(2))
        else:
            hdr, d = None, 0
        out.append((name, hdr, d, ins))
        i = j
    return out


def count(asm_path: str) -> dict:
    lines = open(asm_path).read().split("\n")
    res = {}
    for key, prefix in KERNELS.items():
        st = next(i for i, l in enumerate(lines) if l.startswith(prefix))
        en = next(i for i in range(st, len(lines)) if lines[i].startswith(".Lfunc_end"))
        blocks = _blocks(lines[st:en])
        hot = max((b for b in blocks if b[1]), key=lambda b: sum("row_bcast:31" in x for x in b[3]))
        sel = [b for b in blocks if b[1] == hot[1] and b[2] == hot[2]
               and not any(x.startswith("v_rndne_f64") for x in b[3])]
        c = Counter()
        for b in sel:
            c.update(x.split()[0] for x in b[3] if x.startswith("v_"))
        res[key] = {
            "valu_per_round": sum(c.values()),
            "transcendental": sum(v for k, v in c.items()
                                  if any(t in k for t in ("log", "exp", "sqrt", "sin", "cos", "rcp", "rsq"))),
            "int32_mul": sum(v for k, v in c.items() if "mul_hi_u32" in k or "mul_lo_u32" in k or "mad_u64" in k),
            "f64": sum(v for k, v in c.items() if "f64" in k),
            "blocks": len(sel),
        }
    return res


def main() -> None:
    with tempfile.TemporaryDirectory() as d:
        s = os.path.join(d, "dmb.s")
        assemble(s)
        for k, v in count(s).items():
            print(k, v)


if __name__ == "__main__":
    sys.exit(main())
