"""The C-ABI library loads and exports every symbol include/rm.h declares (CPU only:
no compute call is made without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2412_08076_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(rm_\w+)\s*\(", text, flags=re.M)))


def test_header_declarations_are_bound():
    decl = declared_functions()
    assert len(decl) >= 15
    assert sorted(_lib.EXPORTS) == decl


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librm.so not built (python -m paper_2412_08076_amd.build)")
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (rm_\w+)$", out, flags=re.M))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert hasattr(lib, f)


def test_host_only_entry_points(lib):
    assert lib.rm_meta_param_count(16) == 5457
    assert lib.rm_status_string(0) == b"ok"
    assert lib.rm_status_string(1) == b"invalid argument"
    # argument errors are caught on the host before any HIP call
    h = ctypes.c_void_p()
    inst = (_lib.rm_instance * 1)()
    inst[0].n, inst[0].op, inst[0].eps = 8, 0, 0.5
    assert lib.rm_plan(None, 1, inst, None, ctypes.byref(h)) == _lib.RM_EINVAL
    assert lib.rm_create(None, 0, None) == _lib.RM_EINVAL
    opts = _lib.rm_solve_opts()
    assert lib.rm_solve(None, None, 1, ctypes.byref(opts), None, None, None, None, None, None, None) == \
        _lib.RM_EINVAL
    assert b"null" in lib.rm_last_error()
    assert lib.rm_plan_points(None) == -1
    # kernel-configuration calls reject a null plan before touching it
    sh, T, cw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.rm_plan_set_kernel(None, 0, 9, 8, 0) == _lib.RM_EINVAL
    assert lib.rm_plan_set_tail_kernel(None, 0, 0, 8, 0) == _lib.RM_EINVAL
    assert lib.rm_plan_get_tail_kernel(None, 255, ctypes.byref(sh), ctypes.byref(T), ctypes.byref(cw)) == \
        _lib.RM_EINVAL
    assert lib.rm_plan_set_tail_switch(None, 0.5) == _lib.RM_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of every struct in include/rm.h, compiled by gcc, equal
    the ctypes declarations of the binding."""
    structs = {
        "rm_instance": _lib.rm_instance,
        "rm_solve_opts": _lib.rm_solve_opts,
        "rm_report": _lib.rm_report,
        "rm_fgmres_opts": _lib.rm_fgmres_opts,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)
