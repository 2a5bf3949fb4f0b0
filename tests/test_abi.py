"""The C ABI: the built library loads here (no GPU needed), exports every
function include/dfpr.h declares, and the binding's struct layouts match
the header as a C compiler sees it.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfpr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfpr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_19562_amd import dfpr
    if not os.path.exists(dfpr.LIB_PATH):
        from paper_2407_19562_amd import build
        build.build()
    return dfpr


def test_header_declares_the_binding_names(lib):
    assert declared_functions() == sorted(lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    handle = lib._lib()
    for name in declared_functions():
        assert hasattr(handle, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (dfpr_\w+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_header(lib, tmp_path):
    prog = tmp_path / "layout.c"
    fields_p = [f for f, _ in lib.dfpr_params._fields_]
    fields_s = [f for f, _ in lib.dfpr_stats._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
             "int main(void){",
             'printf("%zu %zu\\n", sizeof(dfpr_params), sizeof(dfpr_stats));']
    for f in fields_p:
        lines.append(f'printf("%zu\\n", offsetof(dfpr_params, {f}));')
    for f in fields_s:
        lines.append(f'printf("%zu\\n", offsetof(dfpr_stats, {f}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(prog)], check=True)
    vals = subprocess.run([str(exe)], capture_output=True, text=True,
                          check=True).stdout.split()
    sp, ss = int(vals[0]), int(vals[1])
    assert sp == ctypes.sizeof(lib.dfpr_params)
    assert ss == ctypes.sizeof(lib.dfpr_stats)
    offs = list(map(int, vals[2:]))
    want = [getattr(lib.dfpr_params, f).offset for f in fields_p] + \
           [getattr(lib.dfpr_stats, f).offset for f in fields_s]
    assert offs == want


def test_defaults_follow_the_paper(lib):
    p = lib.dfpr_params_default()
    assert p.alpha == 0.85 and p.tol == 1e-10 and p.max_iters == 500
    assert p.frontier_tol == pytest.approx(p.tol / 1000)
    assert p.precision == 64


def test_strerror_and_bad_params(lib):
    assert lib.dfpr_strerror(lib.DFPR_EINVAL) == "invalid argument"
    h = lib._lib()
    # create with n <= 0 is rejected before any device call
    out = ctypes.c_void_p()
    assert h.dfpr_graph_create(0, 0, None, None, 0, None, None,
                               ctypes.byref(out)) == lib.DFPR_EINVAL
    assert "n must be > 0" in lib.dfpr_last_error()
    p = lib.dfpr_params_default(alpha=1.5)
    assert h.dfpr_graph_create(4, 0, None, None, 0, ctypes.byref(p), None,
                               ctypes.byref(out)) == lib.DFPR_EINVAL


def test_null_graph_is_rejected(lib):
    # every graph entry point checks its handle before any device call
    h = lib._lib()
    for name, args in [("dfpr_add_vertices", (1, None)),
                       ("dfpr_remove_vertices", (1,)),
                       ("dfpr_mark_reachable", (None,)),
                       ("dfpr_update_traversal", (None,)),
                       ("dfpr_update", (None,)),
                       ("dfpr_set_faults", (None, 0))]:
        assert getattr(h, name)(None, *args) == lib.DFPR_EINVAL, name
        assert "NULL" in lib.dfpr_last_error()


@pytest.mark.parametrize("field,value", [
    ("chunk", 32), ("chunk", 100), ("chunk", 8192), ("block_size", 96),
    ("block_size", 512), ("reorder", 3), ("split_min_degree", -1),
    ("kahan_min_degree", -1), ("max_iters", 0), ("max_iters", 9000),
    ("precision", 16), ("grid_blocks", 1 << 20), ("timeout_ms", -5),
    ("graph_replay", 3)])
def test_invalid_parameters_are_rejected_before_any_device_call(lib, field, value):
    h = lib._lib()
    out = ctypes.c_void_p()
    p = lib.dfpr_params_default(**{field: value})
    assert h.dfpr_graph_create(4, 0, None, None, 0, ctypes.byref(p), None,
                               ctypes.byref(out)) == lib.DFPR_EINVAL
    assert field.split("_")[0] in lib.dfpr_last_error()


def test_automatic_chunk_and_grid_are_valid(lib):
    # chunk, grid_blocks and block_size 0 (the defaults) pass validation: on a host
    # without a device the call fails later, with a device error
    h = lib._lib()
    out = ctypes.c_void_p()
    p = lib.dfpr_params_default()
    assert p.chunk == 0 and p.grid_blocks == 0 and p.block_size == 0
    rc = h.dfpr_graph_create(4, 0, None, None, 0, ctypes.byref(p), None, ctypes.byref(out))
    assert rc != lib.DFPR_EINVAL
    if rc == lib.DFPR_OK:
        h.dfpr_graph_destroy(out)
