"""Sampled oracle checks at full lattice size.

The operators are local: the output at a site x depends only on input and
links within a fixed hop distance R of x (R = 0 for the fifth-dimension
operators, 1 for dslash_eo, 4 for D_PC^+ D_PC and its block restriction).  A
window of extent 2R + 2 per dimension around x, cut out of the full lattice and
treated as a small periodic lattice, therefore holds everything the output at
x depends on, with no path able to wrap around the window within R hops.  The
oracle runs on that small lattice; its output at x is compared with the GPU's
output at x on the full lattice, computed in the launch configuration the
solvers use.

Inputs are sparse so that nothing of full size is built on the host: random
spinors on the sites within R of each sample, zero elsewhere; random SU(3)
links within R + 1 of each sample, unit links elsewhere.  The time boundary
sign of the full lattice is folded into its boundary links before they are
copied into a window, and the window itself is periodic.

Nothing here is imported by the GPU library or by the oracle.
"""
from __future__ import annotations

import numpy as np

from paper_1811_08488_amd import synth


def lex_of(L, c):
    c = np.asarray(c)
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def coords_of(L, lex):
    lex = np.asarray(lex)
    out = np.empty(lex.shape + (4,), np.int64)
    r = lex.copy()
    for mu in range(4):
        out[..., mu] = r % L[mu]
        r = r // L[mu]
    return out


def ball(L, x, R):
    """Lex indices of the sites within L1 hop distance R of coordinate x (periodic)."""
    offs = [o for o in np.ndindex(*(2 * R + 1,) * 4) if sum(abs(v - R) for v in o) <= R]
    c = (np.asarray(x)[None, :] + np.asarray(offs) - R) % np.asarray(L)[None, :]
    return np.unique(lex_of(L, c))


class Window:
    """A periodic sub-lattice around x whose origin o keeps x R or R + 1 sites
    from its lower edge, with extent 2R + 2 (or the full extent where that is
    smaller); sum(o) is even so that every site keeps its parity.

    `pins` maps a dimension to a full-lattice block boundary B (the first
    coordinate of a block) that x sits next to (x = B - 1 or B): the window
    then puts B at its midpoint E/2, so that splitting the window into two
    blocks in that dimension reproduces the cut at B (and the window's own
    periodic seam stays more than R hops from x).  Where the parity has to be
    fixed and every shortened dimension is pinned, one pinned extent grows by
    two."""

    def __init__(self, L, x, R, pins=None):
        self.L = tuple(L)
        pins = pins or {}
        E, o = [], []
        for mu in range(4):
            if L[mu] <= 2 * R + 4 and mu not in pins:
                E.append(L[mu])
                o.append(0)
            elif mu in pins:
                E.append(2 * R + 2)
                o.append(pins[mu] - (R + 1))
            else:
                E.append(2 * R + 2)
                o.append(x[mu] - R)
        if sum(o) % 2:
            free = [mu for mu in range(4) if E[mu] < L[mu] and mu not in pins]
            if free:
                o[free[0]] -= 1
            else:
                mu = sorted(pins)[0]
                E[mu] += 2
                o[mu] -= 1
        self.E, self.o = tuple(E), np.asarray(o)
        off = (np.asarray(x) - self.o) % np.asarray(L)
        for mu in range(4):
            if E[mu] < L[mu]:
                assert R <= off[mu] <= E[mu] - 1 - R, "sample too close to the window seam"
        self.V = int(np.prod(E))
        self.full_lex = lex_of(L, (coords_of(E, np.arange(self.V)) + self.o) % np.asarray(L))

    def sub_lex(self, full_coord):
        return int(lex_of(self.E, (np.asarray(full_coord) - self.o) % np.asarray(self.L)))

    def gauge(self, Ufull, tbc):
        """Window links: the full lattice's, with the time boundary sign folded in."""
        U = np.array(Ufull[self.full_lex])
        t = coords_of(self.L, self.full_lex)[:, 3]
        U[t == self.L[3] - 1, 3] *= tbc
        return U

    def field(self, parity, cb_full, values):
        """Window cb field [V/2, ...] of `parity` from sparse full-lattice values at cb_full (sorted)."""
        sub = np.arange(self.V)
        c = coords_of(self.E, sub)
        sub = sub[(c.sum(-1) % 2) == parity]
        full_cb = self.full_lex[sub] >> 1
        out = np.zeros((self.V // 2,) + values.shape[1:], values.dtype)
        pos = np.searchsorted(cb_full, full_cb)
        pos = np.minimum(pos, len(cb_full) - 1)
        hit = cb_full[pos] == full_cb
        out[sub[hit] >> 1] = values[pos[hit]]
        return out


class SparseLattice:
    """Unit links with random SU(3) patches around the sample sites, and sparse
    random input fields; everything seeded."""

    def __init__(self, L, samples, R, eps, seed):
        self.L = tuple(L)
        self.V = int(np.prod(L))
        rng = np.random.default_rng(seed)
        U = np.zeros((self.V, 4, 3, 3), np.complex128)
        U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
        patch = np.unique(np.concatenate([ball(L, x, R + 1) for x in samples]))
        U[patch] = synth.random_su3(len(patch) * 4, eps, rng).reshape(len(patch), 4, 3, 3)
        self.U = U
        self.rng = rng

    def sparse_input(self, samples, R, parity, Ls, nrhs):
        """cb indices (sorted) of the sites of `parity` within R of a sample, and
        random values [n, nrhs, Ls, 4, 3] on them."""
        sites = np.unique(np.concatenate([ball(self.L, x, R) for x in samples]))
        c = coords_of(self.L, sites)
        sites = sites[(c.sum(-1) % 2) == parity]
        cb = np.sort(sites >> 1)
        vals = (self.rng.standard_normal((len(cb), nrhs, Ls, 4, 3, 2)) @ np.array([1.0, 1j])) / np.sqrt(2.0)
        return cb, vals


def sample_sites(L, parity, n_random, seed, extra=()):
    """Corner sites (wrapping in every direction, crossing the time boundary),
    `extra` coordinates and seeded random ones, each moved onto `parity`."""
    rng = np.random.default_rng(seed)
    pts = [np.zeros(4, np.int64), np.asarray(L) - 1] + [np.asarray(e) for e in extra]
    pts += [rng.integers(0, np.asarray(L)) for _ in range(n_random)]
    out = []
    for p in pts:
        p = np.array(p) % np.asarray(L)
        if p.sum() % 2 != parity:
            p[0] = (p[0] + 1) % L[0]
        out.append(p)
    return out
