"""The C-ABI library loads on the CPU and exports every entry point declared in include/wbfbt.h;
host-only entry points (mesh metadata, options, argument checks) work without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wbfbt.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"WB_API\s+[\w\s\*]+?\b(wb_\w+)\s*\(", src)))


def _lib():
    from paper_1607_03936_amd import wbfbt
    if not os.path.exists(wbfbt.LIB_PATH):
        pytest.fail("libwbfbt.so is not built (run __graft_entry__.build())")
    return wbfbt, wbfbt.lib()


def test_header_declares_the_boundary():
    names = declared()
    for must in ["wb_mesh_create", "wb_visc_create_sinker", "wb_rhs_sinker", "wb_apply_A",
                 "wb_apply_B", "wb_apply_BT", "wb_apply_wbfbt", "wb_solver_create", "wb_solve"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    wb, L = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", wb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (wb_\w+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(L, n)                       # resolvable through ctypes
        assert n in wb.SIGNATURES, f"binding lacks {n}"


def test_host_entry_points_without_gpu():
    wb, L = _lib()
    o = wb.opts()
    assert (o.cheb_degree, o.lanczos_steps, o.restart, o.max_iter, o.rtol) == (3, 10, 100, 1000, 1e-6)
    assert (o.a_l, o.a_r, o.precond_prec) == (1.0, 1.0, wb.WB_FP64)
    m = wb.Mesh(32, 2)
    assert (m.n_nodes, m.n_elem, m.n_p) == (65 ** 3, 32 ** 3, 4)
    m = wb.Mesh(64, 3)
    assert (m.u_len, m.p_len) == (21567171, 2621440)
    h = ctypes.c_void_p()
    assert L.wb_mesh_create(0, 2, ctypes.byref(h)) == wb.WB_EINVAL
    assert b"N must be" in L.wb_last_error()
    assert L.wb_mesh_create(8, 6, ctypes.byref(h)) == wb.WB_EUNSUPPORTED
    m = wb.Mesh(4, 5)
    assert (m.n_nodes, m.n_p) == (21 ** 3, 35)
    assert L.wb_mesh_create(1025, 1, ctypes.byref(h)) == wb.WB_EINVAL
    assert L.wb_apply_A(None, None, None, None, None) == wb.WB_EINVAL
    assert L.wb_solve(None, None, None, None, None, None) == wb.WB_EINVAL


def test_opts_struct_matches_header():
    """The binding's wb_opts mirrors the header's field order and types, and the defaults of the
    later options (graph replay, Schur sign and approximation, assembly limit, weights)."""
    wb, L = _lib()
    src = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} wb_opts;", src, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int|double)\s+([\w\s,]+);", body)
    names = []
    for ty, decl in fields:
        for nm in decl.split(","):
            names.append((nm.strip(), ty))
    ct = {"int": ctypes.c_int, "double": ctypes.c_double}
    assert [(n, ct[t]) for n, t in names] == list(wb.wb_opts._fields_)
    o = wb.opts()
    assert (o.use_graph, o.schur_sign, o.schur_approx, o.weights) == (1, -1, 0, 0)
    assert o.assemble_mb == 32.0
    with pytest.raises(TypeError):
        wb.opts(no_such_option=1)
