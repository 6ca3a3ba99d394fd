"""Full-size parity on sampled sites for every workload (lattice, Ls, nrhs,
action and blocking of the benchmarked configurations), through the C ABI in
the launch configuration the solvers use (tuned workgroup shapes, tile-ordered
sites, halo-extended block domains).  The oracle recomputes each sampled output
on a small periodic window cut around the site (tests/embedding.py).

Tolerances are the per-application ones: FP64 1e-13, FP32 1e-6, FP16/BF16 with
per-site norm 5e-3, as a relative 2-norm over all sampled outputs against the
oracle on the FP64 input and, for the single-hop and fifth-dimension
operators, element by element against each sampled 5D site's norm against
the oracle on the rounded input the kernels read.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import mspcg as M
from paper_1811_08488_amd.workloads import WORKLOADS
from tests import embedding as E
from tests.gpu_util import PNAME, SITE_TOL, TOL, rel, require_gpu, site_err

pytestmark = pytest.mark.gpu

RMAX = 4    # hop range of D_PC^+ D_PC
EPS = 0.45  # width of the random links in the patches


def block_starts(L, n):
    q, rr = divmod(L, n)
    return [j * q + min(j, rr) for j in range(n)] + [L]


def boundary_samples(w):
    """Even sites next to block boundaries: one next to a cut in all four
    dimensions, one next to the cuts in x and t with y, z deep inside a block
    (where the block is long enough).  Returns (coords, pins) pairs."""
    if w.nblk is None:
        return []
    out = []
    for dims in ((0, 1, 2, 3), (0, 3)):
        x, pins = [], {}
        for mu in range(4):
            st = block_starts(w.L[mu], w.nblk[mu])
            size = st[2] - st[1] if w.nblk[mu] >= 2 else w.L[mu]
            if w.nblk[mu] >= 2 and (mu in dims or size < 10):
                pins[mu] = st[1]
                x.append(st[1] - (mu % 2))
            else:
                x.append(st[1] + 5 if w.nblk[mu] >= 2 else w.L[mu] // 2)
        x = np.array(x)
        if x.sum() % 2:  # move onto the even parity: the other side of a cut, or one site along x
            if pins:
                mu = min(pins)
                x[mu] = pins[mu] if x[mu] == pins[mu] - 1 else pins[mu] - 1
            else:
                x[0] += 1
        out.append((x, pins))
    return out


@pytest.fixture(scope="module", params=list(WORKLOADS), ids=list(WORKLOADS))
def W(request):
    torch = require_gpu()
    w = WORKLOADS[request.param]
    s0 = E.sample_sites(w.L, 0, 2, seed=w.gauge_seed)
    s1 = E.sample_sites(w.L, 1, 2, seed=w.gauge_seed + 7)
    bs = boundary_samples(w)
    lat = E.SparseLattice(w.L, s0 + s1 + [x for x, _ in bs], RMAX, EPS, seed=w.gauge_seed + 11)
    h = M.Handle(M.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c, t_bc=-1), lat.U)
    yield SimpleNamespace(w=w, h=h, lat=lat, samples={0: s0, 1: s1}, bs=bs)
    h.close()
    torch.cuda.empty_cache()


def sub_action(w, win):
    return O.Action(win.E, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c, tbc=1.0)


def gpu_input(S, cb, vals, parity, prec):
    f = S.h.field(M.F64, S.w.nrhs, parity)
    S.h.write_sites(f, cb, vals.transpose(1, 0, 2, 3, 4))
    if prec == M.F64:
        return f
    g = S.h.field(prec, S.w.nrhs, parity)
    S.h.convert(g, f)
    return g


def rounded_vals(S, f, cb):
    """The input values a field holds at the sparse sites cb, as [n, nrhs, Ls, 4, 3]."""
    return S.h.read_sites(f, cb).transpose(1, 0, 2, 3, 4)


def oracle_at(S, x, R, in_parity, cb, vals, fn, pins=None):
    """[nrhs, Ls, 4, 3]: fn(sub_action, sub_links, sub_input, window) at x on its window."""
    w = S.w
    win = E.Window(w.L, x, R, pins)
    Asub, Usub = sub_action(w, win), win.gauge(S.lat.U, -1.0)
    out = []
    for r in range(w.nrhs):
        psi = win.field(in_parity, cb, vals[:, r])
        out.append(fn(Asub, Usub, psi, win)[win.sub_lex(x) >> 1])
    return np.stack(out)


def cb_of(L, pts):
    return np.array([int(E.lex_of(L, p)) >> 1 for p in pts])


@pytest.mark.parametrize("prec", [M.F64, M.F32, M.F16, M.BF16], ids=lambda p: PNAME[p])
@pytest.mark.parametrize("dagger", [0, 1])
def test_dslash_eo_sampled(W, prec, dagger):
    S = W
    for p in (0, 1):
        pts = S.samples[p]
        cb, vals = S.lat.sparse_input(pts, 1, 1 - p, S.w.Ls, S.w.nrhs)
        fin = gpu_input(S, cb, vals, 1 - p, prec)
        out = S.h.field(prec, S.w.nrhs, p)
        S.h.dslash_eo(out, fin, dagger)
        got = S.h.read_sites(out, cb_of(S.w.L, pts))

        def op(A, U, psi, win):
            return O.dslash_eo(A, U, psi, p, dagger)

        want = np.stack([oracle_at(S, x, 1, 1 - p, cb, vals, op) for x in pts], axis=1)
        assert rel(got, want) <= TOL[prec], (p, rel(got, want))
        rv = rounded_vals(S, fin, cb)
        want_r = np.stack([oracle_at(S, x, 1, 1 - p, cb, rv, op) for x in pts], axis=1)
        assert site_err(got, want_r) <= SITE_TOL[prec], (p, site_err(got, want_r))


@pytest.mark.parametrize("dagger", [0, 1])
def test_m5inv_sampled(W, dagger):
    S = W
    pts = S.samples[1]
    cb, vals = S.lat.sparse_input(pts, 0, 1, S.w.Ls, S.w.nrhs)
    out = S.h.field(M.F64, S.w.nrhs, 1)
    S.h.m5inv(out, gpu_input(S, cb, vals, 1, M.F64), dagger)
    got = S.h.read_sites(out, cb_of(S.w.L, pts))
    which = 3 if dagger else 2
    want = np.stack([oracle_at(S, x, 0, 1, cb, vals, lambda A, U, psi, win: O.op5(A, psi, which, 1))
                     for x in pts], axis=1)
    assert rel(got, want) <= TOL[M.F64]


@pytest.mark.parametrize("prec", [M.F64, M.F32, M.F16], ids=lambda p: PNAME[p])
def test_mdagm_sampled(W, prec):
    S = W
    pts = S.samples[0]
    cb, vals = S.lat.sparse_input(pts, RMAX, 0, S.w.Ls, S.w.nrhs)
    out = S.h.field(prec, S.w.nrhs, 0)
    S.h.mdagm(out, gpu_input(S, cb, vals, 0, prec))
    got = S.h.read_sites(out, cb_of(S.w.L, pts))
    want = np.stack([oracle_at(S, x, RMAX, 0, cb, vals, lambda A, U, psi, win: O.mdagm(A, U, psi)) for x in pts],
                    axis=1)
    assert rel(got, want) <= TOL[prec]


@pytest.mark.parametrize("prec", [M.F64, M.F32, M.F16, M.BF16], ids=lambda p: PNAME[p])
def test_block_apply_sampled(W, prec):
    """Sites next to block cuts (snake terms, uneven splits)."""
    S = W
    if S.w.nblk is None:
        pytest.skip("plain CG workload: no blocks")
    pts = [x for x, _ in S.bs]
    cb, vals = S.lat.sparse_input(pts, RMAX, 0, S.w.Ls, S.w.nrhs)
    out = S.h.field(M.F64, S.w.nrhs, 0)
    S.h.block_apply(out, gpu_input(S, cb, vals, 0, M.F64), S.w.nblk, prec)
    got = S.h.read_sites(out, cb_of(S.w.L, pts))
    want = []
    for x, pins in S.bs:
        nsub = [2 if mu in pins else 1 for mu in range(4)]

        def blk_op(A, U, psi, win, nsub=nsub, x=x):
            blk = int(O.block_of_site(win.E, nsub)[win.sub_lex(x)])
            return O.block_op(A, U, psi, nsub, blk)

        want.append(oracle_at(S, x, RMAX, 0, cb, vals, blk_op, pins))
    want = np.stack(want, axis=1)
    assert rel(got, want) <= TOL[prec]
