"""The C-ABI library loads and exports every symbol include/dmb.h declares
(no GPU needed: no compute call is made)."""
import os
import re
import subprocess

import pytest

import paper_2603_24688_amd as dmb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "dmb.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(dmb_[a-z_]+)\s*\(", src, re.M)))


def test_header_declares_binding_exports():
    assert declared_symbols() == sorted(dmb.EXPORTS)


@pytest.mark.skipif(not os.path.exists(dmb.LIB_PATH), reason="libdmb.so not built")
def test_library_exports_all_symbols():
    L = dmb.load_library()
    for s in declared_symbols():
        assert hasattr(L, s), s
    nm = subprocess.run(["nm", "-D", "--defined-only", dmb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (dmb_\w+)", nm))
    assert set(declared_symbols()) <= exported


def test_library_is_gfx950_code_object():
    if not os.path.exists(dmb.LIB_PATH):
        pytest.skip("libdmb.so not built")
    blob = open(dmb.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(dmb.DmbError):
        dmb._lib_backup = dmb._lib
        try:
            dmb._lib = None
            dmb.load_library(str(tmp_path / "missing.so"))
        finally:
            dmb._lib = dmb._lib_backup


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU only: --gpus 2 exits with a message (no GPU needed)."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
