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
    assert (o.mode, o.tau, o.wg_size, o.blocks_per_cu, o.timeout_ms) == (0, 0, 1024, 1, 20000)


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the size and field offsets that a C compiler
    gives the structs of include/pasgal.h."""
    import subprocess
    from paper_2404_17101_amd import _lib as L
    mirrors = {"pasgal_csr": L.Csr, "pasgal_opts": L.Opts, "pasgal_stats": L.Stats, "pasgal_scc_opts": L.SccOpts,
               "pasgal_scc_stats": L.SccStats, "pasgal_batch_desc": L.BatchDesc,
               "pasgal_server_opts": L.ServerOpts, "pasgal_request": L.Request, "pasgal_completion": L.Completion}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pasgal.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_new_entry_points_reject_bad_arguments_on_the_host(lib):
    """Argument checks happen before any HIP call, so they run without a GPU."""
    from paper_2404_17101_amd import _lib as L
    L._lib = None
    lib = L.load()
    P = ctypes.POINTER
    csr = L.Csr(0, 0, None, None)  # n = 0 is invalid
    out = ctypes.c_void_p(1)
    assert lib.pasgal_scc(ctypes.byref(csr), None, out, None, None, None) == -1
    assert lib.pasgal_sssp(ctypes.byref(csr), None, 0, out, None, None) == -1
    assert lib.pasgal_bfs_do(ctypes.byref(csr), None, 0, out, 0, 0, None, None) == -1
    good = L.Csr(4, 0, ctypes.c_void_p(1), None)
    # SCC: unknown flag bits and a transpose of another size are rejected
    so = L.SccOpts(-1, 0x80, 0, 0)
    assert lib.pasgal_scc(ctypes.byref(good), None, out, ctypes.byref(so), None, None) == -1
    other = L.Csr(5, 0, ctypes.c_void_p(1), None)
    assert lib.pasgal_scc(ctypes.byref(good), ctypes.byref(other), out, None, None, None) == -1
    # sources out of range, missing output
    assert lib.pasgal_sssp(ctypes.byref(good), None, 4, out, None, None) == -1
    assert lib.pasgal_bfs_do(ctypes.byref(good), None, -1, out, 0, 0, None, None) == -1
    assert lib.pasgal_bfs_do(ctypes.byref(good), None, 0, None, 0, 0, None, None) == -1
    # latency probe: null result, sizes, step counts and kinds out of range
    ns = ctypes.c_double(-1.0)
    assert lib.pasgal_probe_latency(1 << 20, 100, 0, None, None) == -1
    assert lib.pasgal_probe_latency(4095, 100, 0, ctypes.byref(ns), None) == -1
    assert lib.pasgal_probe_latency((1 << 32) + 1, 100, 0, ctypes.byref(ns), None) == -1
    assert lib.pasgal_probe_latency(1 << 20, 0, 0, ctypes.byref(ns), None) == -1
    assert lib.pasgal_probe_latency(1 << 20, (1 << 24) + 1, 0, ctypes.byref(ns), None) == -1
    assert lib.pasgal_probe_latency(1 << 20, 100, 3, ctypes.byref(ns), None) == -1
    assert lib.pasgal_probe_latency(1 << 20, 100, -1, ctypes.byref(ns), None) == -1
    assert ns.value == -1.0
    # the no-allocation BFS: bad arguments, and a graph beyond the vertices its
    # fixed device array can serve, are rejected before anything runs
    assert lib.pasgal_bfs_noalloc(ctypes.byref(csr), 0, out, None, None) == -1
    assert lib.pasgal_bfs_noalloc(ctypes.byref(good), 4, out, None, None) == -1
    assert lib.pasgal_bfs_noalloc(ctypes.byref(good), 0, None, None, None) == -1
    huge = L.Csr((1 << 28) + 1, 0, ctypes.c_void_p(1), None)
    assert lib.pasgal_bfs_noalloc(ctypes.byref(huge), 0, out, None, None) == -5
    ao = L.Opts()
    lib.pasgal_opts_default(ctypes.byref(ao))
    ao.flags = L.FLAG_ASYNC
    assert lib.pasgal_bfs_noalloc(ctypes.byref(good), 0, out, ctypes.byref(ao), None) == -1
    # defaults of the VGC options
    o = L.Opts()
    lib.pasgal_opts_default(ctypes.byref(o))
    assert (o.heavy_arcs, o.filter_slots, o.window) == (512, 256, 0)


def test_constants_match_header():
    """The binding's flag, mode and request constants carry the values that
    include/pasgal.h defines."""
    from paper_2404_17101_amd import _lib as L
    txt = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define PASGAL_(\w+) \(?(-?\d+)u?\)?", txt)}
    checked = 0
    for name, val in defs.items():
        if name.startswith(("FLAG_", "MODE_", "REQ_", "SCC_", "BATCH_", "SERVER_")):
            assert getattr(L, name) == val, name
            checked += 1
    assert checked >= 12
    for code, text in L.ERRORS.items():
        assert defs[text] == code, (code, text)
