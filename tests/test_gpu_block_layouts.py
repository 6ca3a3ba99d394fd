"""GPU parity of the batched block CG and the MSPCG solve on every lane layout
of the inner kernels, against the FP64 CPU oracle.

The kernels pick their layout from Ls and the number of right-hand sides:
one DPP row per (site, rhs) column for Ls = 16; whole columns per 64-lane
wave with ds_bpermute exchanges for Ls dividing 64 (Ls = 8) and for Ls = 12
with one right-hand side (block lists padded to 320 sites); densely packed
columns with LDS exchanges for Ls = 24 and for Ls = 12 with 8 right-hand
sides.  Each layout is run with FP64 inner storage (which must reproduce the
oracle's textbook CG up to rounding, so any indexing slip in the gather,
update, per-block scalar or scatter kernels shows) and with the storage types
the workloads use.  Lattices include 16 blocks and an uneven split.

Comparisons are element by element against the norm of each 5D site
(tests.gpu_util.site_err).  Low-precision inner solves: k iterations whose
operator applications each carry the per-application error e (5e-3 for
FP16/BF16 storage, 1e-6 for FP32) and whose vectors are rounded to the
storage type at every update; the error of the k-step result relative to the
site norm is bounded here by 2 k e (the iteration is a fixed polynomial in
A_s of degree k - 1 applied to r, with coefficients that depend smoothly on
the same perturbed inner products).
"""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import mspcg as M
from tests.gpu_util import PNAME, Setup, rel, require_gpu, site_err

pytestmark = pytest.mark.gpu

# id: (L, Ls, nblk, nrhs)
LAYOUTS = {
    "dpp_ls16_16blocks": ((8, 8, 8, 8), 16, (2, 2, 2, 2), 1),
    "wave_ls12_16blocks": ((8, 8, 8, 8), 12, (2, 2, 2, 2), 1),
    "lds_ls12_rhs8": ((4, 4, 4, 8), 12, (1, 1, 1, 2), 8),
    "lds_ls24": ((4, 4, 4, 8), 24, (1, 1, 1, 2), 1),
    "bpermute_ls8_uneven": ((10, 8, 6, 12), 8, (3, 2, 1, 2), 1),
}
# per-application error of the inner operator in each storage type
APP_ERR = {M.F32: 1e-6, M.F16: 5e-3, M.BF16: 5e-3}


@pytest.fixture(scope="module", params=list(LAYOUTS), ids=list(LAYOUTS))
def LY(request):
    require_gpu()
    L, Ls, nblk, nrhs = LAYOUTS[request.param]
    s = Setup(L, Ls, "mobius", mf=0.05, seed=21)
    s.nblk, s.nrhs, s.name = nblk, nrhs, request.param
    return s


def _oracle_z(S, r, k, rhs_list):
    return {i: O.local_block_cg(S.oa, S.U, r[i], S.nblk, k) for i in rhs_list}


def _checked_rhs(S):
    return [0, S.nrhs - 1] if S.nrhs > 1 else [0]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_local_block_cg_f64_every_layout(LY, k):
    S = LY
    r = S.rand(S.nrhs, 300 + k)
    fz = S.h.field(M.F64, S.nrhs, 0)
    S.h.local_block_cg(fz, S.h.upload(r, 0), S.nblk, k, M.F64)
    got = S.h.download(fz)
    for i, want in _oracle_z(S, r, k, _checked_rhs(S)).items():
        assert site_err(got[i], want) <= 1e-10, (S.name, k, i, site_err(got[i], want))


@pytest.mark.parametrize("prec", [M.F32, M.F16, M.BF16], ids=lambda p: PNAME[p])
def test_local_block_cg_low_precision_every_layout(LY, prec):
    S, k = LY, 3
    r = S.rand(S.nrhs, 310)
    fz = S.h.field(M.F64, S.nrhs, 0)
    S.h.local_block_cg(fz, S.h.upload(r, 0), S.nblk, k, prec)
    got = S.h.download(fz)
    for i, want in _oracle_z(S, r, k, _checked_rhs(S)).items():
        err = site_err(got[i], want)
        print(f"[block-cg] {S.name} {PNAME[prec]} k={k} rhs={i}: site err {err:.3e}, rel {rel(got[i], want):.3e}")
        assert err <= 2 * k * APP_ERR[prec], (S.name, PNAME[prec], i, err)


def test_block_apply_every_layout(LY):
    """One application of the direct sum of the A_s (FP64 storage) on each layout."""
    S = LY
    x = S.rand(S.nrhs, 320)
    fout = S.h.field(M.F64, S.nrhs, 0)
    S.h.block_apply(fout, S.h.upload(x, 0), S.nblk, M.F64)
    got = S.h.download(fout)
    nb = int(np.prod(S.nblk))
    for i in _checked_rhs(S):
        want = sum(O.block_op(S.oa, S.U, x[i], S.nblk, b) for b in range(nb))
        assert site_err(got[i], want) <= 1e-12, (S.name, i, site_err(got[i], want))


# solves on lattices small enough for the oracle's literal preconditioner
# (one whole-lattice A per block and inner iteration): id -> (L, Ls, nblk, nrhs)
SOLVES = {
    "dpp_ls16": ((4, 4, 4, 8), 16, (1, 1, 1, 2), 1),
    "wave_ls12": ((4, 4, 4, 8), 12, (1, 1, 1, 2), 2),
    "lds_ls12_rhs8": ((4, 4, 4, 8), 12, (1, 1, 1, 2), 8),
    "lds_ls24": ((4, 4, 4, 8), 24, (1, 1, 1, 2), 1),
    "bpermute_ls8_uneven": ((4, 4, 4, 14), 8, (1, 1, 1, 3), 1),
}


@pytest.mark.parametrize("case", list(SOLVES), ids=list(SOLVES))
def test_mspcg_solve_every_layout(case):
    require_gpu()
    L, Ls, nblk, nrhs = SOLVES[case]
    S = Setup(L, Ls, "mobius", mf=0.05, seed=22)
    b = S.rand(nrhs, 330)
    checked = [0, nrhs - 1] if nrhs > 1 else [0]
    # FP64 inner storage: the oracle's Algorithm 1 iterates
    fx = S.h.field(M.F64, nrhs, 0)
    st = S.h.mspcg_solve(fx, S.h.upload(b, 0), nblk, 3, M.F64, tol=1e-10)
    x = S.h.download(fx)
    assert st["status"] == M.OK
    for i in checked:
        xo, st_o = O.solve(S.oa, S.U, b[i], nblk=nblk, k=3, tol=1e-10, maxiter=2000)
        assert site_err(x[i], xo) <= 1e-7, (case, i, site_err(x[i], xo))
        assert abs(st["outer_iters"] - st_o.iters) <= 2 + 0.02 * st_o.iters
    # FP16 inner storage: converges to the same solution, true residual recomputed by the oracle
    fx = S.h.field(M.F64, nrhs, 0)
    st = S.h.mspcg_solve(fx, S.h.upload(b, 0), nblk, 3, M.F16, tol=1e-10)
    x = S.h.download(fx)
    assert st["status"] == M.OK
    for i in checked:
        res = np.linalg.norm(b[i] - O.mdagm(S.oa, S.U, x[i])) / np.linalg.norm(b[i])
        assert res <= 1e-10, (case, i, res)
