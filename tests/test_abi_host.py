"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol that include/mspcg.h declares, and rejects invalid arguments before any
device work with the documented status."""
import ctypes
import os
import re

import pytest

from paper_1811_08488_amd import mspcg as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mspcg.h")).read()
    return re.findall(r"^(?:mspcg_status|const char \*)\s*(\w+)\(", src, flags=re.M)


def test_header_declares_the_boundary():
    names = set(declared_functions())
    for required in ("dslash_eo", "m5inv", "mdagm", "local_block_cg", "mspcg_solve", "cg_solve"):
        assert required in names
    assert names == set(M.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = M.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C
    compiler gives the header's structs (a field added on one side only would
    shift every later field)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mspcg_dwf": M.Dwf, "mspcg_field": M.CField, "mspcg_precond": M.Precond,
               "mspcg_solver": M.Solver, "mspcg_stats": M.Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mspcg.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def _dwf(**kw):
    d = dict(L=(4, 4, 4, 4), Ls=8, M5=1.8, mf=0.01, b=1.0, c=0.0, t_bc=-1)
    d.update(kw)
    return M.Dwf((ctypes.c_int * 4)(*d["L"]), d["Ls"], d["M5"], d["mf"], d["b"], d["c"], d["t_bc"])


@pytest.mark.parametrize(
    "kw,status",
    [
        (dict(L=(4, 4, 3, 4)), M.EINVAL),
        (dict(L=(4, 0, 4, 4)), M.EINVAL),
        (dict(Ls=1), M.EINVAL),
        (dict(Ls=64), M.EUNSUPPORTED),
        (dict(t_bc=0), M.EINVAL),
        (dict(M5=float("nan")), M.EINVAL),
    ],
)
def test_create_rejects_bad_parameters(kw, status):
    h = ctypes.c_void_p()
    gauge = (ctypes.c_double * 8)()  # never dereferenced: validation fails first
    rc = M.lib().mspcg_create(ctypes.byref(h), ctypes.byref(_dwf(**kw)), ctypes.cast(gauge, ctypes.c_void_p), None)
    assert rc == status
    assert h.value is None
    assert M.lib().mspcg_last_error().decode() != ""


def test_null_arguments():
    L = M.lib()
    assert L.mspcg_create(None, None, None, None) == M.EINVAL
    f = M.CField(None, None, 0, 1, 0)
    assert L.dslash_eo(None, ctypes.byref(f), ctypes.byref(f), 0, None) == M.EINVAL
    assert L.mdagm(None, ctypes.byref(f), ctypes.byref(f), None) == M.EINVAL
    assert L.m5inv(None, ctypes.byref(f), ctypes.byref(f), 0, None) == M.EINVAL
    assert L.cg_solve(None, ctypes.byref(f), ctypes.byref(f), None, None) == M.EINVAL
    assert L.mspcg_solve(None, ctypes.byref(f), ctypes.byref(f), None, None, None) == M.EINVAL
    assert L.local_block_cg(None, ctypes.byref(f), ctypes.byref(f), None, None) == M.EINVAL
    assert L.mspcg_destroy(None) == M.OK
