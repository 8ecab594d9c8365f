"""The C-ABI library loads and exports every symbol include/dotpe.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2507_16022_amd import dotpe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "dotpe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dotpe_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(dotpe.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dotpe.SYMBOLS), "binding and header disagree"


def test_version_and_error_string():
    lib = dotpe.load_library()
    assert lib.dotpe_version().startswith(b"dotpe")
    assert isinstance(lib.dotpe_last_error(), bytes)


def test_struct_layouts():
    # sizes must match the C structs (checked against hand-computed layouts)
    assert ctypes.sizeof(dotpe.BankDesc) == 8 + 4 + 4 + 5 * 8 + 4 + 4
    assert ctypes.sizeof(dotpe.Sample) == 32
    assert ctypes.sizeof(dotpe.EvidenceResult) == 7 * 8 + 3 * 8 + 4 * 4 + 2 * 8
