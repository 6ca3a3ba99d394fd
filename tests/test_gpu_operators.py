"""GPU parity of the operators (through the C ABI) against the FP64 CPU oracle.

Sizes span several workgroup tiles and a ragged last tile; index work is
compared bit-exactly, floating point within the per-application tolerance
(FP64 1e-13, FP32 1e-6, FP16/BF16 with per-site norm 5e-3): over the whole
field against the oracle on the FP64 input, and element by element against
the norm of each 5D site against the oracle on the rounded input the kernels
read (operators made of n stored stages: n times the per-application bound).
"""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import mspcg as M
from tests import lattice_helpers as H
from tests.gpu_util import PNAME, PRECS, SITE_TOL, TOL, Setup, rel, require_gpu, rounded, site_err

pytestmark = pytest.mark.gpu

LATTICES = [((8, 8, 8, 8), 8), ((6, 4, 2, 10), 12)]


@pytest.fixture(scope="module", params=LATTICES, ids=lambda p: "x".join(map(str, p[0])) + f"_ls{p[1]}")
def S(request):
    require_gpu()
    L, Ls = request.param
    return Setup(L, Ls, "mobius", seed=3)


@pytest.fixture(scope="module")
def S_shamir():
    require_gpu()
    return Setup((8, 4, 4, 6), 8, "shamir", seed=4)


@pytest.mark.parametrize("parity", [0, 1])
def test_site_maps_bit_exact(S, parity):
    lex, nbr = S.h.site_maps(parity)
    olex, onbr = O.site_maps(S.L, parity)
    assert np.array_equal(lex, olex)
    assert np.array_equal(nbr, onbr)


@pytest.mark.parametrize("L,nblk,block", [((8, 8, 8, 8), (2, 2, 2, 2), 5), ((10, 8, 6, 12), (3, 2, 1, 2), 7),
                                          ((10, 8, 6, 12), (3, 2, 1, 2), 0)])
def test_block_domains_match_brute_force(L, nblk, block):
    require_gpu()
    s = Setup(L, 4, "mobius", seed=5)
    be, o1, e2 = s.h.block_sites(nblk, block)
    bBe, bO1, bE2 = H.halo_sets_bfs(L, nblk, block)
    assert sorted(be.tolist()) == bBe and sorted(o1.tolist()) == bO1 and sorted(e2.tolist()) == bE2
    assert len(set(e2.tolist())) == len(e2) and len(set(o1.tolist())) == len(o1)
    # B_e is in block-local lexicographic order
    c = H.coords_of_lex(L)[be]
    key = [tuple(reversed(((cc - c.min(0)) % np.array(L)).tolist())) for cc in c]
    assert key == sorted(key)
    # the oracle's block membership agrees
    blk = O.block_of_site(L, nblk)
    assert np.all(blk[be] == block)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PNAME[p])
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_eo(S, prec, dagger, out_parity):
    nrhs = 2 if prec == M.F64 else 1
    x = S.rand(nrhs, 10 + dagger + 2 * out_parity)
    fin = S.h.upload(x, 1 - out_parity, prec)
    fout = S.h.field(prec, nrhs, out_parity)
    S.h.dslash_eo(fout, fin, dagger)
    got = S.h.download(fout)
    xr = rounded(S.h, x, 1 - out_parity, prec)
    for r in range(nrhs):
        want = O.dslash_eo(S.oa, S.U, x[r], out_parity, dagger)
        assert rel(got[r], want) <= TOL[prec], (PNAME[prec], r, rel(got[r], want))
        want_r = O.dslash_eo(S.oa, S.U, xr[r], out_parity, dagger)
        assert site_err(got[r], want_r) <= SITE_TOL[prec], (PNAME[prec], r, site_err(got[r], want_r))


@pytest.mark.parametrize("prec", [M.F16, M.BF16], ids=lambda p: PNAME[p])
@pytest.mark.parametrize("L,Ls", [((4, 4, 4, 4), 16), ((4, 4, 4, 6), 12), ((4, 4, 2, 4), 24)],
                         ids=["dpp_ls16", "bpermute_ls12", "lds_ls24"])
def test_dslash_eo_half_precision_wide_norm_range(L, Ls, prec):
    """Inputs whose magnitude swings by up to four orders between neighbouring
    s (and one all-zero slice): the per-site norms and the rescaled M_phi
    mixing keep every output slice within the per-application tolerance of
    its own magnitude (no overflow, no loss of the small slices)."""
    require_gpu()
    S = Setup(L, Ls, "mobius", seed=6)
    prof = 10.0 ** (3.0 * np.sin(1.3 * np.arange(Ls) + 0.4))
    prof[Ls // 3] = 0.0
    x = S.rand(1, 50) * prof[None, None, :, None, None]
    for dagger in (0, 1):
        fout = S.h.field(prec, 1, 0)
        S.h.dslash_eo(fout, S.h.upload(x, 1, prec), dagger)
        got = S.h.download(fout)[0]
        want = O.dslash_eo(S.oa, S.U, x[0], 0, dagger)
        for s in range(Ls):
            assert np.all(np.isfinite(got[:, s]))
            assert rel(got[:, s], want[:, s]) <= TOL[prec], (PNAME[prec], dagger, s, rel(got[:, s], want[:, s]))


def test_dslash_eo_shamir(S_shamir):
    S = S_shamir
    x = S.rand(1, 20)
    for dagger in (0, 1):
        fin = S.h.upload(x, 1)
        fout = S.h.field(M.F64, 1, 0)
        S.h.dslash_eo(fout, fin, dagger)
        assert rel(S.h.download(fout)[0], O.dslash_eo(S.oa, S.U, x[0], 0, dagger)) <= 1e-13


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PNAME[p])
@pytest.mark.parametrize("dagger", [0, 1])
def test_m5inv(S, prec, dagger):
    x = S.rand(1, 30 + dagger)
    fin = S.h.upload(x, 0, prec)
    fout = S.h.field(prec, 1, 0)
    S.h.m5inv(fout, fin, dagger)
    got = S.h.download(fout)[0]
    which = O.M5INV_DAG if dagger else O.M5INV
    assert rel(got, O.op5(S.oa, x[0], which, 0)) <= TOL[prec]
    want_r = O.op5(S.oa, rounded(S.h, x, 0, prec)[0], which, 0)
    assert site_err(got, want_r) <= SITE_TOL[prec], site_err(got, want_r)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PNAME[p])
def test_mdagm(S, prec):
    nrhs = 2 if prec == M.F64 else 1
    x = S.rand(nrhs, 40)
    fin = S.h.upload(x, 0, prec)
    fout = S.h.field(prec, nrhs, 0)
    S.h.mdagm(fout, fin)
    got = S.h.download(fout)
    xr = rounded(S.h, x, 0, prec)
    for r in range(nrhs):
        want = O.mdagm(S.oa, S.U, x[r])
        assert rel(got[r], want) <= TOL[prec], (PNAME[prec], rel(got[r], want))
        # four hops, each with a stored (rounded) output
        want_r = O.mdagm(S.oa, S.U, xr[r])
        assert site_err(got[r], want_r) <= 4 * SITE_TOL[prec], (PNAME[prec], site_err(got[r], want_r))


def test_mdagm_shamir(S_shamir):
    S = S_shamir
    x = S.rand(1, 41)
    fout = S.h.field(M.F64, 1, 0)
    S.h.mdagm(fout, S.h.upload(x, 0))
    assert rel(S.h.download(fout)[0], O.mdagm(S.oa, S.U, x[0])) <= 1e-13


def _oracle_block_sum(S, x, nblk, truncated=False):
    nb = int(np.prod(nblk))
    return sum(O.block_op(S.oa, S.U, x, nblk, b, truncated) for b in range(nb))


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PNAME[p])
@pytest.mark.parametrize("L,Ls,nblk", [((8, 8, 8, 8), 8, (2, 2, 2, 2)), ((10, 8, 6, 12), 4, (3, 2, 1, 2))])
def test_block_apply(L, Ls, nblk, prec):
    require_gpu()
    S = Setup(L, Ls, "mobius", seed=6)
    x = S.rand(1, 50)
    fout = S.h.field(M.F64, 1, 0)
    S.h.block_apply(fout, S.h.upload(x, 0), nblk, prec)
    got = S.h.download(fout)[0]
    want = _oracle_block_sum(S, x[0], nblk)
    assert rel(got, want) <= TOL[prec], (PNAME[prec], rel(got, want))
    # the input is gathered into `prec` (rounded) and passes four stored hops
    want_r = _oracle_block_sum(S, rounded(S.h, x, 0, prec)[0], nblk)
    assert site_err(got, want_r) <= 4 * SITE_TOL[prec], (PNAME[prec], site_err(got, want_r))


@pytest.mark.parametrize("prec", [M.F64, M.F32], ids=lambda p: PNAME[p])
@pytest.mark.parametrize("L,Ls,nblk", [((8, 8, 8, 8), 8, (2, 2, 2, 2)), ((10, 8, 6, 12), 4, (3, 2, 1, 2))])
def test_block_apply_without_snake_terms(L, Ls, nblk, prec):
    """Every hop cut at the block boundary (the variant Sec. 2.3 compares against)."""
    require_gpu()
    S = Setup(L, Ls, "mobius", seed=6)
    x = S.rand(1, 51)
    fout = S.h.field(M.F64, 1, 0)
    S.h.block_apply(fout, S.h.upload(x, 0), nblk, prec, no_snake=1)
    got = S.h.download(fout)[0]
    want = _oracle_block_sum(S, x[0], nblk, truncated=True)
    assert rel(got, want) <= TOL[prec]
    # and it differs from the operator with the snake terms
    assert rel(got, _oracle_block_sum(S, x[0], nblk)) > 1e-3


def test_prepare_and_reconstruct(S):
    rng = np.random.default_rng(7)
    V = int(np.prod(S.L))
    phi = H.rand_c(rng, (V, S.Ls, 4, 3))
    b_o, _ = O.prepare_rhs(S.oa, S.U, phi)
    phi_e, phi_o = H.full_to_cb(S.L, phi, 0), H.full_to_cb(S.L, phi, 1)
    fb = S.h.field(M.F64, 1, 0)
    fe, fo = S.h.upload(phi_e, 0), S.h.upload(phi_o, 1)
    S.h.prepare_rhs(fb, fe, fo)
    assert rel(S.h.download(fb)[0], b_o) <= 1e-13
    psi_e = H.rand_c(rng, (V // 2, S.Ls, 4, 3))
    full = O.reconstruct(S.oa, S.U, psi_e, phi)
    fpo = S.h.field(M.F64, 1, 1)
    S.h.reconstruct(fpo, S.h.upload(psi_e, 0), fo)
    assert rel(S.h.download(fpo)[0], H.full_to_cb(S.L, full, 1)) <= 1e-13


def test_conversions_round_trip(S):
    x = S.rand(1, 60)
    for prec, tol in ((M.F32, 1e-7), (M.F16, 1e-3), (M.BF16, 8e-3)):
        back = S.h.download(S.h.upload(x, 0, prec))
        assert rel(back, x) <= tol
    # an all-zero site survives the per-site norm
    x[0, 3] = 0
    back = S.h.download(S.h.upload(x, 0, M.F16))
    assert np.all(back[0, 3] == 0) and np.isfinite(back).all()


def test_create_rejects_zero_b():
    """The hop kernels factor b out of M_phi = b + c P_chi: b = 0 is refused at create."""
    require_gpu()
    from paper_1811_08488_amd import synth

    L = (4, 4, 4, 4)
    with pytest.raises(M.MspcgError) as e:
        M.Handle(M.Action(L, 4, M5=1.8, mf=0.1, b=0.0, c=0.5), synth.gauge_field(L, 0.3, 1))
    assert e.value.status == M.EUNSUPPORTED
