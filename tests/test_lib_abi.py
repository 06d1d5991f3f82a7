"""The C-ABI library loads on the CPU host and exports every symbol the header declares
(no compute calls: there is no GPU here).  Host-side argument checks return errors
before anything is launched."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2404_13216_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pbicgstab.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[a-z_0-9]+\s*\**\s+)+\**([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_parsed():
    names = declared_symbols()
    assert "pbicgstab_solve" in names and "exdot" in names and "csr_spmv" in names


def test_all_declared_symbols_exported():
    L = pk.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(pk.EXPORTS) <= set(declared_symbols())


def _c_layout(tmp_path):
    """sizeof / offsetof of every field, printed by a C program compiled against the header."""
    structs = {"pbcg_csr": pk.PbcgCsr, "pbcg_opts": pk.PbcgOpts, "pbcg_info": pk.PbcgInfo,
               "pbcg_vectors": pk.PbcgVectors, "pbcg_sliced": pk.PbcgSliced}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pbicgstab.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True)
    return structs, {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_struct_layout_matches_header(tmp_path):
    structs, lay = _c_layout(tmp_path)
    for cname, py in structs.items():
        assert lay[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert lay[(cname, f)] == getattr(py, f).offset, (cname, f)
    assert pk.lib().pbcg_abi_version() == 8


def test_status_strings_and_defaults():
    assert pk.status_string(0) == "ok"
    assert pk.status_string(-4) == "workspace too small"
    o = pk.default_opts()
    assert o.tol == 1e-10 and o.max_iter == 10000 and o.batch == 16 and o.inner_tol == 0.1 and o.max_outer == 60


def test_host_argument_checks_without_gpu():
    L = pk.lib()
    # null matrix / negative sizes are rejected before any launch
    assert L.csr_spmv(None, None, None, None) == pk.ERR_INVALID
    assert L.exdot(-1, None, None, None, None, 0, None) == pk.ERR_INVALID
    out = ctypes.c_double()
    assert L.exdot(0, None, None, ctypes.byref(out), None, 0, None) == pk.ERR_WORKSPACE
    assert L.exdot_config(4, None, None, None, 1, 256, 4, None, 0, None) == pk.ERR_INVALID
    bad = pk.PbcgCsr(-1, 0, 0, None, None, None)
    o = pk.default_opts()
    assert L.pbicgstab_solve(ctypes.byref(bad), None, None, ctypes.byref(o), None, None, 0, None) == pk.ERR_INVALID
    good = pk.PbcgCsr(4, 0, 4, 1, 1, 1)  # fake non-null pointers: never dereferenced on the host
    assert L.pbicgstab_solve(ctypes.byref(good), 1, 1, ctypes.byref(o), None, None, 0, None) == pk.ERR_WORKSPACE
    o.tol = -1.0
    assert L.pbicgstab_solve(ctypes.byref(good), 1, 1, ctypes.byref(o), None, 256, 1 << 20, None) == pk.ERR_INVALID
    # kernel timing events: a multiple of 8, with an array
    o = pk.default_opts()
    o.kernel_events_len = 4
    assert L.pbicgstab_solve(ctypes.byref(good), 1, 1, ctypes.byref(o), None, 256, 1 << 20, None) == pk.ERR_INVALID
    o.kernel_events_len = 8
    assert L.pbicgstab_solve(ctypes.byref(good), 1, 1, ctypes.byref(o), None, 256, 1 << 20, None) == pk.ERR_INVALID
    # sliced copies: bad matrix, missing workspace, unbuilt copy
    S = pk.PbcgSliced()
    assert L.csr_slice(None, ctypes.byref(S), None, 0, None) == pk.ERR_INVALID
    assert L.csr_slice(ctypes.byref(good), None, None, 0, None) == pk.ERR_INVALID
    assert L.csr_slice(ctypes.byref(good), ctypes.byref(S), None, 0, None) == pk.ERR_WORKSPACE
    assert L.csr_slice(ctypes.byref(good), ctypes.byref(S), 256, 16, None) == pk.ERR_WORKSPACE
    assert L.csr_spmv_sliced(ctypes.byref(good), ctypes.byref(S), 8, 16, None) == pk.ERR_INVALID
    assert L.csr_spmv_sliced(ctypes.byref(good), None, 8, 16, None) == pk.ERR_INVALID
    assert L.csr_spmv_f32_sliced(ctypes.byref(good), ctypes.byref(S), 8, 16, None) == pk.ERR_INVALID  # F64 values


def test_workspace_sizes_monotone():
    L = pk.lib()
    o = pk.default_opts()
    a = L.pbicgstab_workspace_bytes(1000, 5000, ctypes.byref(o))
    b = L.pbicgstab_workspace_bytes(100000, 500000, ctypes.byref(o))
    assert b > a >= 12 * 1000 * 8
    o.prec = pk.PREC_FP32_IR
    c = L.pbicgstab_workspace_bytes(100000, 500000, ctypes.byref(o))
    assert c >= b + 11 * 100000 * 4 + 500000 * 4
    # the sliced copy (layout AUTO, the default): 12 bytes per entry of nnz + nnz/8 + 256
    o.prec = pk.PREC_FP64
    o.layout = pk.LAYOUT_CSR
    d = L.pbicgstab_workspace_bytes(100000, 500000, ctypes.byref(o))
    assert b - d >= 12 * (500000 + 500000 // 8 + 256) + 8 * (100000 // 256 + 1)
    o.spmv_kind, o.layout = pk.SPMV_VECTOR, pk.LAYOUT_AUTO     # only the row-sequential kernels slice
    assert L.pbicgstab_workspace_bytes(100000, 500000, ctypes.byref(o)) == d
    assert L.csr_slice_workspace_bytes(100000, 500000) >= 12 * (500000 + 500000 // 8 + 256)
    assert L.csr_slice_workspace_bytes(-1, 0) == 0
