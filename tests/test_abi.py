"""The C-ABI library loads and exports every entry point include/msz.h declares (no GPU needed)."""
import os
import re
import subprocess

import pytest

import paper_2406_09423_amd as msz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "msz.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msz_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("msz_fix", "msz_labels", "msz_count_false", "msz_fix_batch", "msz_workspace_bytes",
                 "msz_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(msz.LIB_PATH):
        pytest.fail("libmsz.so is not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", msz.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (msz_[a-z_]+)\b", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    lib = msz.lib()
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_host_only_entry_points():
    assert msz.strerror(msz.OK) == "ok"
    assert msz.strerror(msz.EBOUND).startswith("error bound")
    n = 3600 * 2400
    wb = msz.workspace_bytes((2400, 3600))
    assert wb >= 29 * n and wb < 30 * n   # L, g, 2 dirs, marks, case bytes, dirty flags, 4 int32 label/pointer arrays
    assert msz.workspace_bytes((1, 1)) > 0
    assert msz.lib().msz_workspace_bytes(msz.Dims(2, 4, 4, 2)) == 0      # 2D with nz != 1
    assert msz.lib().msz_workspace_bytes(msz.Dims(3, 0, 4, 4)) == 0
    # vertex counts up to 2^31 - 2^16 (sizes rounded up to whole chunks stay in 32 bits)
    assert msz.lib().msz_workspace_bytes(msz.Dims(2, 2 ** 15 - 1, 2 ** 16, 1)) > 0   # exactly the limit
    assert msz.lib().msz_workspace_bytes(msz.Dims(2, 2 ** 15, 2 ** 16 - 1, 1)) == 0  # 2^15 above it
    assert msz.lib().msz_workspace_bytes(msz.Dims(2, 2 ** 31 - 1, 1, 1)) == 0
    assert msz.lib().msz_workspace_bytes(msz.Dims(3, 1291, 1291, 1291)) == 0
    assert msz.lib().msz_workspace_bytes(msz.Dims(3, 2048, 2048, 512)) == 0   # n >= 2^31
    assert msz.tile_variants(2) >= 1 and msz.tile_variants(3) >= 1
    both = msz.workspace_bytes((64, 80)) + msz.workspace_bytes((16, 16, 16))
    assert msz.batch_workspace_bytes([(64, 80), (16, 16, 16)]) == both   # the fields' own workspaces


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus N > 1 exits with status 2 and says why
    before touching a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
