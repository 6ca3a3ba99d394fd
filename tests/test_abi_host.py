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
