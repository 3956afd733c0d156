"""The C-ABI library loads and exports every entry point of include/lsbdg.h
(CPU only: no compute call is made)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2511_05233_amd import lsbdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsbdg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lsbdg.LIB_PATH):
        pytest.fail("liblsbdg.so is not built (run __graft_entry__.build())")
    return lsbdg.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    assert sorted(lsbdg.exported_symbols()) == _declared()


def test_default_parameters_are_the_papers(lib):
    """dg_params_default fills Tab. 5 (host-only call)."""
    p = lsbdg.default_params()
    assert p.T == 298.15
    assert list(p.D0) == [9.3e-10, 10.0e-10, 5.3e-10, 5.3e-10, 7.6e-10, 0.6e-10, 9.3e-10]
    assert list(p.kE) == [2.53e-6, 3.54e-8, 1.49e-10, 2.05e-7, 9.11e-10, 1.37e-15]
    assert p.use_TH == 1


def test_struct_layouts_match_the_header():
    assert ctypes.sizeof(lsbdg.DgMesh) == 24
    assert ctypes.sizeof(lsbdg.DgParams) == 8 * (1 + 7 + 6 + 6) + 8


_STRUCTS = {"dg_mesh": lsbdg.DgMesh, "dg_params": lsbdg.DgParams, "dg_solver_opts": lsbdg.DgSolverOpts,
            "dg_step_report": lsbdg.DgStepReport, "dg_controller": lsbdg.DgController,
            "dg_advance_report": lsbdg.DgAdvanceReport, "dg_batch_shape": lsbdg.DgBatchShape,
            "dg_batch_tuning": lsbdg.DgBatchTuning}


def test_binding_structs_match_the_c_compiler(tmp_path):
    """sizeof and every field offset of the ctypes structures equal what a C
    compiler makes of include/lsbdg.h."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lsbdg.h"', "int main(void) {"]
    for cname, cls in _STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, cls in _STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_batch_setup_rejects_bad_arguments(lib):
    """Both failures are found before any device call."""
    import numpy as np
    out = ctypes.c_void_p()
    assert lib.dg_batch_setup(0, None, None, None, ctypes.byref(out)) == -1
    mesh = (lsbdg.DgMesh * 2)(lsbdg.DgMesh(2, 2, 2, 1, 1e-6), lsbdg.DgMesh(2, 2, 2, 1, 1e-6))
    params = (lsbdg.DgParams * 2)(lsbdg.default_params(), lsbdg.default_params())
    bad = np.full(8, 2, np.uint8)
    ptrs = (ctypes.c_void_p * 2)(bad.ctypes.data, bad.ctypes.data)
    assert lib.dg_batch_setup(2, mesh, ptrs, params, ctypes.byref(out)) == -1
    assert b"structure 0" in lib.dg_last_error()
    ptrs = (ctypes.c_void_p * 2)(None, bad.ctypes.data)
    assert lib.dg_batch_setup(2, mesh, ptrs, params, ctypes.byref(out)) == -1
    assert b"null phase map of structure 0" in lib.dg_last_error()
    assert not out.value


def test_batch_shape_calls_reject_bad_arguments(lib):
    """Null batches and reports are refused before any device call."""
    sh = lsbdg.DgBatchShape(32, 0)
    assert lib.dg_batch_set_shape(None, 0, 0, ctypes.byref(sh)) == -1
    assert lib.dg_batch_get_shape(None, 0, 0, ctypes.byref(sh)) == -1
    rep = lsbdg.DgBatchTuning()
    assert lib.dg_batch_autotune(None, 0, None, None, None, None, None, None, 5, ctypes.byref(rep), None) == -1
    assert b"null argument" in lib.dg_last_error()


def test_binding_constants_match_the_header_enums():
    """Every enumerator of include/lsbdg.h equals the binding's constant
    (status codes through the binding's name table)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    enums = {}
    for body in re.findall(r"typedef\s+enum\s*\w*\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(DG_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            enums[name] = int(val)
    assert len(enums) == 26, sorted(enums)   # status 8, precision 2, JVP 3, controller 2, batch op 3, workspace 8
    for name, val in enums.items():
        if hasattr(lsbdg, name):
            assert getattr(lsbdg, name) == val, name
        else:
            assert lsbdg._STATUS[val] == name, name


def test_orders_and_workspace_sizes_are_checked_on_the_host(lib):
    """Orders outside {0, 1, 3} are invalid, order 0 provides the operators
    only and order 3 the operators and element blocks; the workspace of the operator entry points holds the
    phase map, the status flag, the FP64 linearisation (14 values per node)
    and the output partial sums, each 256-byte aligned."""
    import ctypes as C
    p = lsbdg.default_params()
    ph = (C.c_uint8 * 8)(*([1] * 8))
    out = C.c_void_p()
    for order in (2, -1, 4):
        mesh = lsbdg.DgMesh(2, 2, 2, order, 1e-6)
        assert lib.dg_setup(C.byref(mesh), ph, C.byref(p), C.byref(out)) == -1, order
    n = C.c_size_t()
    mesh3 = lsbdg.DgMesh(3, 2, 2, 3, 1e-6)
    assert lib.dg_workspace_bytes(C.byref(mesh3), C.byref(p), None, lsbdg.DG_WS_STEP, C.byref(n)) == -7
    assert lib.dg_workspace_bytes(C.byref(mesh3), C.byref(p), None, lsbdg.DG_WS_OPERATORS, C.byref(n)) == 0
    al = lambda x: (x + 255) // 256 * 256
    assert n.value == al(al(al(al(12) + 4) + 14 * 12 * 64 * 8) + 15 * 1024 * 8)
    # order 3 also sizes its element blocks (FP32 448 x 448 inverses, the
    # pivot lists and two FP32 7-field probe vectors)
    feats = lsbdg.DG_WS_OPERATORS | lsbdg.DG_WS_BLOCKS
    assert lib.dg_workspace_bytes(C.byref(mesh3), C.byref(p), None, feats, C.byref(n)) == 0
    ops = al(al(al(12) + 4) + 14 * 12 * 64 * 8) + 15 * 1024 * 8
    assert n.value == al(al(al(al(ops) + 12 * 448 * 448 * 4) + 12 * 448 * 2) + 14 * 12 * 64 * 4)
    mesh = lsbdg.DgMesh(96, 96, 192, 1, 1e-6)
    assert lib.dg_workspace_bytes(C.byref(mesh), C.byref(p), None, 128, C.byref(n)) == -1   # unknown bit
    # the multigrid workspace needs explicit levels; bad solver options are
    # refused before any device call
    assert lib.dg_workspace_bytes(C.byref(mesh), C.byref(p), None, lsbdg.DG_WS_MG, C.byref(n)) == -1
    for field, bad in (("mg_levels", 1), ("mg_levels", 9), ("mg_levels", -2), ("mg_sweeps", 9), ("mg_omega", 0.0),
                       ("mg_omega", 1.5), ("block_reuse", -1.0), ("coarse_agg", -1), ("coarse", 5)):
        o = lsbdg._solver_opts("f32", {field: bad})
        assert lib.dg_workspace_bytes(C.byref(mesh), C.byref(p), C.byref(o), lsbdg.DG_WS_OPERATORS,
                                      C.byref(n)) == -1, (field, bad)
    o = lsbdg._solver_opts("f32", {})
    assert (o.mg_levels, o.mg_sweeps, o.mg_omega, o.block_reuse, o.coarse) == (-1, 3, 0.7, 1.0, 0)
    assert lib.dg_workspace_bytes(C.byref(mesh), C.byref(p), None, lsbdg.DG_WS_OPERATORS, C.byref(n)) == 0
    al = lambda x: (x + 255) // 256 * 256
    Ne = 96 * 96 * 192
    expect = al(al(al(Ne) + 4) + 14 * Ne * 8 * 8) + 15 * 1024 * 8
    assert n.value == al(expect), (n.value, expect)
    mesh0 = lsbdg.DgMesh(4, 4, 4, 0, 1e-6)
    assert lib.dg_workspace_bytes(C.byref(mesh0), C.byref(p), None, lsbdg.DG_WS_STEP, C.byref(n)) == -7


def test_triad_rejects_bad_arguments_on_the_host(lib):
    """dg_triad refuses a negative length and null arrays, and n = 0 is a
    no-op, all before any device call."""
    assert lib.dg_triad(None, None, None, 1.0, 0, None) == 0
    assert lib.dg_triad(None, None, None, 1.0, -2, None) == -1
    assert lib.dg_triad(None, None, None, 1.0, 4, None) == -1
