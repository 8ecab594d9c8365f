"""The C-ABI library loads and exports every symbol include/dotpe.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2507_16022_amd import dotpe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="dotpe.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dotpe_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(dotpe.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 12
    test_names = declared_symbols("dotpe_test.h")
    for n in names + test_names:
        assert hasattr(lib, n), n
    assert set(names) == set(dotpe.SYMBOLS), "binding and header disagree"
    assert set(test_names) == set(dotpe.TEST_SYMBOLS), "binding and test header disagree"


def test_version_and_error_string():
    lib = dotpe.load_library()
    assert lib.dotpe_version().startswith(b"dotpe")
    assert isinstance(lib.dotpe_last_error(), bytes)


def test_struct_layouts():
    # sizes must match the C structs (checked against hand-computed layouts)
    assert ctypes.sizeof(dotpe.BankDesc) == 8 + 4 + 4 + 5 * 8 + 4 + 4 + 4 + 4 + 8
    assert ctypes.sizeof(dotpe.Sample) == 32
    assert ctypes.sizeof(dotpe.EvidenceResult) == 7 * 8 + 3 * 8 + 4 * 4 + 2 * 8 + 8 + 2 * 4 + 8 + 2 * 4 + 3 * 8


STRUCTS = {
    "dotpe_bank_desc": dotpe.BankDesc,
    "dotpe_event_desc": dotpe.EventDesc,
    "dotpe_evidence_result": dotpe.EvidenceResult,
    "dotpe_sample": dotpe.Sample,
    "dotpe_server_desc": dotpe.ServerDesc,
    "dotpe_ticket_info": dotpe.TicketInfo,
    "dotpe_preselect_desc": dotpe.PreselectDesc,
    "dotpe_posterior_sample": dotpe.PosteriorSample,
    "dotpe_preselect_result": dotpe.PreselectResult,
    "dotpe_rb_desc": dotpe.RBDesc,
    "dotpe_extrinsic_desc": dotpe.ExtrinsicDesc,
    "dotpe_extrinsic_result": dotpe.ExtrinsicResult,
}


def test_struct_layouts_match_c_compiler(tmp_path):
    """Every ctypes mirror has the size and field offsets gcc gives the header's structs."""
    import shutil
    import subprocess
    import pytest
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dotpe.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n"):
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
