"""The windows behind the full-size sampled GPU checks are exact: the oracle on
a window around a site reproduces the oracle on the whole lattice at that site
(dslash_eo, its adjoint, D_PC^+ D_PC and the block operator next to block cuts),
with the time boundary sign folded into the window's links."""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd.workloads import Workload
from tests import embedding as E
from tests.test_gpu_full_size import boundary_samples

L, LS = (16, 12, 12, 16), 4
PRM = dict(M5=1.8, mf=0.05, b=1.5, c=0.5)
W = Workload("window_check", L, LS, 1.8, 0.05, 1.5, 0.5, 1, None, (2, 1, 2, 2), 2, "f32")


@pytest.fixture(scope="module")
def setup():
    s0 = E.sample_sites(L, 0, 2, seed=3)
    s1 = E.sample_sites(L, 1, 2, seed=4)
    bs = boundary_samples(W)
    lat = E.SparseLattice(L, s0 + s1 + [x for x, _ in bs], 4, 0.45, seed=5)
    return s0, s1, bs, lat, O.Action(L, LS, **PRM)


def _compare(lat, pts, R, inpar, full_fn, sub_fn, pins=None):
    cb, vals = lat.sparse_input(pts, R, inpar, LS, 1)
    full_in = np.zeros((int(np.prod(L)) // 2, LS, 4, 3), complex)
    full_in[cb] = vals[:, 0]
    full_out = full_fn(full_in)
    for i, x in enumerate(pts):
        win = E.Window(L, x, R, pins[i] if pins else None)
        sub = sub_fn(O.Action(win.E, LS, tbc=1.0, **PRM), win.gauge(lat.U, -1.0), win.field(inpar, cb, vals[:, 0]),
                     win, x)
        want = full_out[int(E.lex_of(L, x)) >> 1]
        assert np.abs(want).max() > 0
        assert np.allclose(sub[win.sub_lex(x) >> 1], want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("dagger", [0, 1])
def test_window_dslash(setup, dagger):
    s0, s1, _, lat, A = setup
    for p, pts in ((0, s0), (1, s1)):
        _compare(lat, pts, 1, 1 - p, lambda f: O.dslash_eo(A, lat.U, f, p, dagger),
                 lambda a, u, f, win, x: O.dslash_eo(a, u, f, p, dagger))


def test_window_mdagm(setup):
    s0, _, _, lat, A = setup
    _compare(lat, s0, 4, 0, lambda f: O.mdagm(A, lat.U, f), lambda a, u, f, win, x: O.mdagm(a, u, f))


def test_window_block_op(setup):
    _, _, bs, lat, A = setup
    pts, pins = [x for x, _ in bs], [p for _, p in bs]
    assert any(len(p) >= 2 for p in pins)
    blk = O.block_of_site(L, W.nblk)

    def full(f):
        out = np.zeros_like(f)
        for x in pts:
            i = int(E.lex_of(L, x))
            out[i >> 1] = O.block_op(A, lat.U, f, W.nblk, int(blk[i]))[i >> 1]
        return out

    def sub(a, u, f, win, x):
        nsub = [2 if mu in dict(zip(map(tuple, pts), pins))[tuple(x)] else 1 for mu in range(4)]
        return O.block_op(a, u, f, nsub, int(O.block_of_site(win.E, nsub)[win.sub_lex(x)]))

    _compare(lat, pts, 4, 0, full, sub, pins)
