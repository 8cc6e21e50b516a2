"""The C-ABI library: it loads and exports every function include/dl.h declares.

No compute call is made here (these tests run without a GPU).
"""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dl.h")
LIB = os.path.join(ROOT, "paper_1608_00139_amd", "libdl.so")


def declared_functions() -> list[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(dl_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dl_create", "dl_destroy", "dl_tc", "dl_sg", "dl_solve_eps", "dl_status_str", "dl_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdl.so not built")
def test_host_only_entry_points():
    import paper_1608_00139_amd as dl

    lib = dl.load()
    assert lib.dl_status_str(0).decode() == "DL_OK"
    assert "invalid" in lib.dl_status_str(1).decode()
    assert dl.dl_padded_size(1, 0) == 256 and dl.dl_padded_size(257, 0) == 512
    assert dl.dl_padded_size(8192, 0) == 8192
    assert dl.dl_padded_size(4, 2) == 128 and dl.dl_padded_size(129, 2) == 256
    assert dl.dl_padded_size(0, 0) == 0


def test_product_path_has_no_fallback():
    """The binding must not import the oracle or carry a CPU path."""
    pkg = os.path.join(ROOT, "paper_1608_00139_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f


def test_tuning_document_round_trip():
    """The autotuner's JSON document: entries survive a round trip; other
    documents and bad entries are rejected (host logic only)."""
    import paper_1608_00139_amd as m

    entries = [{"prec": "i8", "np": 8192, "cfg": 0, "ms": 0.43}, {"prec": "f32", "np": 512, "cfg": 2, "ms": 0.0}]
    text = m.tuning_to_json(entries, "gfx950 test")
    assert m.tuning_from_json(text) == entries
    with pytest.raises(ValueError):
        m.tuning_from_json('{"format": "other", "entries": []}')
    with pytest.raises(ValueError):
        m.tuning_from_json(m.tuning_to_json([{"prec": "f99", "np": 512, "cfg": 0}], "x"))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits at once with a message
    (nothing is imported or launched)."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
