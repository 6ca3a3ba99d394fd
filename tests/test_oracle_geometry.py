"""Pins of the oracle's index maps and block partition against brute force (CPU only)."""
import numpy as np
import pytest

import oracle as O
from tests import lattice_helpers as H


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 8), (8, 8, 8, 8)])
@pytest.mark.parametrize("parity", [0, 1])
def test_site_maps_bijection_and_neighbours(L, parity):
    lex, nbr = O.site_maps(L, parity)
    V = int(np.prod(L))
    c = H.coords_of_lex(L)
    par = c.sum(1) % 2
    # bijection onto the sites of this parity, cb = lex >> 1
    assert sorted(lex.tolist()) == sorted(np.nonzero(par == parity)[0].tolist())
    assert np.array_equal(lex >> 1, np.arange(V // 2))
    # neighbours by brute force on coordinates
    for mu in range(4):
        for d, col in ((1, 0), (-1, 1)):
            y = c[lex].copy()
            y[:, mu] = (y[:, mu] + d) % L[mu]
            ylex = y[:, 0] + L[0] * (y[:, 1] + L[1] * (y[:, 2] + L[2] * y[:, 3]))
            assert np.all(par[ylex] != parity)  # hops flip parity
            assert np.array_equal(nbr[:, mu, col], ylex >> 1)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_neighbour_round_trip(L):
    lex0, nbr0 = O.site_maps(L, 0)
    lex1, nbr1 = O.site_maps(L, 1)
    for mu in range(4):
        fwd = nbr0[:, mu, 0]
        assert np.array_equal(nbr1[fwd, mu, 1], np.arange(len(fwd)))
        bwd = nbr0[:, mu, 1]
        assert np.array_equal(nbr1[bwd, mu, 0], np.arange(len(bwd)))


@pytest.mark.parametrize(
    "L,nblk",
    [((4, 4, 4, 4), (2, 2, 2, 2)), ((32, 32, 32, 8), (3, 3, 3, 4)), ((10, 6, 4, 8), (3, 2, 1, 3)), ((8, 8, 8, 8), (1, 1, 1, 1))],
)
def test_blocks_partition_into_boxes(L, nblk):
    blk = O.block_of_site(L, nblk)
    nb = int(np.prod(nblk))
    assert blk.min() == 0 and blk.max() == nb - 1
    c = H.coords_of_lex(L)
    ranges = H.block_ranges(L, nblk)
    for b in range(nb):
        sel = c[blk == b]
        jb, t = [], b
        for mu in range(4):
            jb.append(t % nblk[mu])
            t //= nblk[mu]
        expect = 1
        for mu in range(4):
            start, size = ranges[mu][jb[mu]]
            assert sel[:, mu].min() == start and sel[:, mu].max() == start + size - 1
            expect *= size
        assert len(sel) == expect  # a full box: the blocks partition the lattice


def test_uneven_extents_32_over_3():
    assert [s for _, s in H.block_ranges((32, 32, 32, 64), (3, 3, 3, 4))[0]] == [11, 11, 10]


@pytest.mark.parametrize("L,nblk,block", [((8, 8, 8, 8), (2, 2, 2, 2), 5), ((8, 6, 8, 10), (2, 1, 2, 2), 3)])
def test_halo_sets_bfs_match_distance(L, nblk, block):
    Be, O1, E2 = H.halo_sets_bfs(L, nblk, block)
    d = H.block_distance(L, nblk, block)
    par = H.parity_of_lex(L)
    assert Be == sorted(np.nonzero((d == 0) & (par == 0))[0].tolist())
    assert O1 == sorted(np.nonzero((d <= 1) & (par == 1))[0].tolist())
    assert E2 == sorted(np.nonzero((d <= 2) & (par == 0))[0].tolist())


@pytest.mark.parametrize(
    "L,nblk,counts",
    [
        ((16, 16, 16, 32), (2, 2, 2, 2), (4096, 7680, 12416)),
        ((24, 24, 24, 64), (2, 2, 2, 4), (13824, 22464, 33120)),
        ((48, 48, 48, 96), (4, 4, 4, 4), (20736, 32832, 47520)),
    ],
)
def test_halo_counts_of_the_workloads(L, nblk, counts):
    d = H.block_distance(L, nblk, 0)
    par = H.parity_of_lex(L)
    got = (int(((d == 0) & (par == 0)).sum()), int(((d <= 1) & (par == 1)).sum()), int(((d <= 2) & (par == 0)).sum()))
    assert got == counts
