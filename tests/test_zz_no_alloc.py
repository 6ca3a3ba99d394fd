"""The allocation-free entry point mdagm_noalloc (for callers that cannot
allocate device memory) against mdagm, through the C ABI: same operator and
kernels, intermediates in the library's fixed per-GPU scratch array.  Two
calls in a row on each precision, the second with a smaller input, then a
second, smaller lattice; the results equal mdagm's bit for bit and the FP64
ones match the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import mspcg as M
from tests.gpu_util import PNAME, PRECS, Setup, rel, require_gpu

pytestmark = pytest.mark.gpu


def _compare(s, prec, nrhs, seed):
    x = s.rand(nrhs, seed)
    fin = s.h.upload(x, 0, prec)
    ref = s.h.field(prec, nrhs, 0)
    s.h.mdagm(ref, fin)  # (also prepares the links of `prec` on the handle)
    got = s.h.field(prec, nrhs, 0)
    s.h.mdagm_noalloc(got, fin)
    g, r = s.h.download(got), s.h.download(ref)
    assert np.array_equal(g, r), (PNAME[prec], nrhs)
    if prec == M.F64:
        for i in range(nrhs):
            want = O.mdagm(s.oa, s.U, x[i])
            assert rel(g[i], want) <= 1e-13


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PNAME[p])
def test_mdagm_noalloc_matches_mdagm(prec):
    require_gpu()
    big = Setup((8, 8, 8, 8), 8, "mobius", seed=40)
    _compare(big, prec, 3, 41)
    _compare(big, prec, 1, 42)  # a smaller input on the same scratch
    small = Setup((4, 4, 4, 6), 12, "mobius", seed=43)
    _compare(small, prec, 2, 44)
    _compare(small, prec, 1, 45)


def test_mdagm_noalloc_first_use_and_limits():
    require_gpu()
    s = Setup((6, 4, 4, 8), 8, "mobius", seed=46)
    x = s.rand(1, 47)
    # FP64 links exist from creation: usable before any other call, with default launch shapes
    out = s.h.field(M.F64, 1, 0)
    s.h.mdagm_noalloc(out, s.h.upload(x, 0))
    assert rel(s.h.download(out)[0], O.mdagm(s.oa, s.U, x[0])) <= 1e-13
    # another precision before the handle prepared its links: refused, nothing written
    out32 = s.h.field(M.F32, 1, 0)
    with pytest.raises(M.MspcgError) as e:
        s.h.mdagm_noalloc(out32, s.h.upload(x, 0, M.F32))
    assert e.value.status == M.EUNSUPPORTED
    assert not out32.data.any()
    # more than the scratch holds: refused before any device work
    big = Setup((16, 16, 16, 16), 16, "mobius", seed=48)
    need = 2 * (big.Vh * 16 * 24 * 8)
    assert need > M.NOALLOC_SCRATCH_BYTES
    fin = big.h.field(M.F64, 1, 0)
    fout = big.h.field(M.F64, 1, 0)
    with pytest.raises(M.MspcgError) as e:
        big.h.mdagm_noalloc(fout, fin)
    assert e.value.status == M.EUNSUPPORTED
