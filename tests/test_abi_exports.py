"""The C-ABI library loads and exports every symbol include/pasgal.h
declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pasgal.h")
LIB = os.path.join(ROOT, "paper_2404_17101_amd", "libpasgal.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pasgal_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2404_17101_amd import build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ["pasgal_bfs", "pasgal_reach", "pasgal_bfs_ex", "pasgal_reach_ex", "pasgal_transpose",
                 "pasgal_batch_create", "pasgal_batch_run", "pasgal_server_submit", "pasgal_server_poll"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pasgal_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert hasattr(lib, n)


def test_binding_lists_match_header():
    from paper_2404_17101_amd import _lib as L
    assert sorted(L.EXPORTS) == declared()


def test_host_only_calls(lib):
    lib.pasgal_strerror.restype = ctypes.c_char_p
    assert lib.pasgal_strerror(0) == b"ok"
    assert lib.pasgal_strerror(-1) == b"invalid argument"
    assert lib.pasgal_version() == 1
    from paper_2404_17101_amd import _lib as L
    o = L.Opts()
    lib.pasgal_opts_default(ctypes.byref(o))
    assert (o.mode, o.tau, o.wg_size, o.blocks_per_cu, o.timeout_ms) == (0, 1024, 1024, 1, 20000)


def test_struct_layouts_match_header():
    from paper_2404_17101_amd import _lib as L
    assert ctypes.sizeof(L.Csr) == 24
    assert ctypes.sizeof(L.Opts) == 48
    assert ctypes.sizeof(L.Stats) == 80
    assert ctypes.sizeof(L.Request) == 4 * 3 + 64 * 4 + 4 + 8 + 8
