"""The C-ABI library loads and exports every function include/scg.h declares
(no GPU needed: only host-side entry points are called)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scg.h")
LIB = os.path.join(ROOT, "paper_1709_04912_amd", "libscg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(scg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libscg.so is not built: run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("scg_plan_create", "scg_plan_destroy", "scg_workspace_bytes",
                     "scg_project", "scg_backproject", "scg_tv", "scg_filter", "scg_solve",
                     "scg_profile", "scg_profile_read", "scg_default_params", "scg_strerror",
                     "scg_plan_get_tuning", "scg_plan_set_tuning", "scg_plan_autotune",
                     "scg_batch_create", "scg_batch_destroy", "scg_batch_submit",
                     "scg_batch_step", "scg_batch_poll", "scg_batch_cancel",
                     "scg_batch_get_stats", "scg_batch_stream"):
        assert required in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(lib, name):
    assert hasattr(lib, name), name


def test_host_only_entry_points(lib):
    lib.scg_strerror.restype = C.c_char_p
    lib.scg_strerror.argtypes = [C.c_int]
    assert lib.scg_strerror(0) and lib.scg_strerror(-1) != lib.scg_strerror(0)
    # null plans are rejected before any device call
    vp = C.c_void_p
    lib.scg_project.argtypes = [vp, C.c_int, vp, vp, vp]
    assert lib.scg_project(None, 0, None, None, None) == -1
    lib.scg_plan_get_tuning.argtypes = [vp, C.c_int, vp]
    assert lib.scg_plan_get_tuning(None, 0, None) == -1
    lib.scg_batch_step.argtypes = [vp, C.c_int]
    assert lib.scg_batch_step(None, 1) == -1
    lib.scg_batch_poll.argtypes = [vp, C.c_uint64, vp]
    assert lib.scg_batch_poll(None, 1, None) == -1
    lib.scg_static_workspace_bytes.restype = C.c_size_t
    assert lib.scg_static_workspace_bytes() == 32 << 20
    lib.scg_solve_static.argtypes = [vp] * 7 + [C.c_int32, vp, C.c_int32, vp]
    assert lib.scg_solve_static(None, None, None, None, None, None, None, 0, None, 0,
                                None) == -1


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the Python binding passes across the C-ABI has the size
    and field offsets that a C compiler gives the declaration in
    include/scg.h (the header compiled as C99 with gcc)."""
    import shutil
    import subprocess
    from paper_1709_04912_amd import scg as b
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [b.scg_geom, b.scg_params, b.scg_report, b.scg_trace_entry, b.scg_kernel_time,
               b.scg_tuning, b.scg_batch_stats]
    lines = ['#include "scg.h"', "#include <stddef.h>", "#include <stdio.h>", "int main(void) {"]
    for cls in structs:
        name = cls.__name__
        lines.append(f'    printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for cls in structs:
        name = cls.__name__
        assert int(got[name]) == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)
