"""Test-side helpers: closed forms, brute-force geometry and dense matrices.

Nothing here is imported by the GPU library or by the oracle.  Everything is
written from the definitions (not from either implementation) so that it can
pin them.
"""
from __future__ import annotations

import itertools

import numpy as np

# ----------------------------------------------------------------- geometry


def coords_of_lex(L):
    """[V, 4] integer coordinates, lex = x + Lx(y + Ly(z + Lz t))."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def parity_of_lex(L):
    return coords_of_lex(L).sum(axis=1) % 2


def cb_to_full(L, cbf, parity):
    """Parity-packed [V/2, ...] -> full [V, ...] lex field (other parity zero)."""
    V = int(np.prod(L))
    full = np.zeros((V,) + cbf.shape[1:], cbf.dtype)
    lex = np.nonzero(parity_of_lex(L) == parity)[0]
    full[lex] = cbf[lex >> 1]
    return full


def full_to_cb(L, full, parity):
    V = int(np.prod(L))
    out = np.zeros((V // 2,) + full.shape[1:], full.dtype)
    lex = np.nonzero(parity_of_lex(L) == parity)[0]
    out[lex >> 1] = full[lex]
    return out


def block_ranges(L, nblk):
    """Per dimension, list of (start, size) of each block."""
    out = []
    for Lm, n in zip(L, nblk):
        q, r = divmod(Lm, n)
        out.append([(j * q + min(j, r), q + (1 if j < r else 0)) for j in range(n)])
    return out


def block_distance(L, nblk, block):
    """L1 distance (periodic) of every lex site from block `block`."""
    rng = block_ranges(L, nblk)
    jb = []
    b = block
    for mu in range(4):
        jb.append(b % nblk[mu])
        b //= nblk[mu]
    c = coords_of_lex(L)
    dist = np.zeros(len(c), np.int64)
    for mu in range(4):
        start, size = rng[mu][jb[mu]]
        x = c[:, mu]
        inside = (x >= start) & (x < start + size)
        d_lo = (start - x) % L[mu]
        d_hi = (x - (start + size - 1)) % L[mu]
        d = np.minimum(d_lo, d_hi)
        dist += np.where(inside, 0, d)
    return dist


def halo_sets_bfs(L, nblk, block):
    """(B_e, O1, E2) lex site lists by breadth-first search on the lattice graph."""
    V = int(np.prod(L))
    c = coords_of_lex(L)
    lex_of = {tuple(v): i for i, v in enumerate(c)}
    dist_in = block_distance(L, nblk, block)
    frontier = set(np.nonzero(dist_in == 0)[0].tolist())
    dist = {s: 0 for s in frontier}
    for step in (1, 2):
        nxt = set()
        for s in frontier:
            x = c[s]
            for mu in range(4):
                for d in (1, -1):
                    y = x.copy()
                    y[mu] = (y[mu] + d) % L[mu]
                    j = lex_of[tuple(y)]
                    if j not in dist:
                        dist[j] = step
                        nxt.add(j)
        frontier = nxt
    par = parity_of_lex(L)
    Be = sorted(s for s, d in dist.items() if d == 0 and par[s] == 0)
    O1 = sorted(s for s, d in dist.items() if d <= 1 and par[s] == 1)
    E2 = sorted(s for s, d in dist.items() if d <= 2 and par[s] == 0)
    assert len(dist) <= V
    return Be, O1, E2


# ----------------------------------------------------------------- spin algebra
# Chiral basis (project convention): g_k = [[0,-i s_k],[i s_k,0]], g_t = [[0,1],[1,0]].
SIGMA = [
    np.array([[0, 1], [1, 0]], complex),
    np.array([[0, -1j], [1j, 0]], complex),
    np.array([[1, 0], [0, -1]], complex),
]


def gammas():
    g = []
    for k in range(3):
        m = np.zeros((4, 4), complex)
        m[:2, 2:] = -1j * SIGMA[k]
        m[2:, :2] = 1j * SIGMA[k]
        g.append(m)
    m = np.zeros((4, 4), complex)
    m[:2, 2:] = np.eye(2)
    m[2:, :2] = np.eye(2)
    g.append(m)
    g5 = np.diag([1, 1, -1, -1]).astype(complex)
    return g, g5


# ----------------------------------------------------------------- 5th dimension, closed forms
def shift_matrix(Ls, mf, up: bool):
    """S+ (up) / S- as Ls x Ls real matrices with the -mf corner."""
    S = np.zeros((Ls, Ls))
    for s in range(Ls):
        if up:
            if s < Ls - 1:
                S[s, s + 1] = 1
            else:
                S[s, 0] = -mf
        else:
            if s > 0:
                S[s, s - 1] = 1
            else:
                S[s, Ls - 1] = -mf
    return S


def chiral_blocks(Ls, M5, mf, b, c):
    """Per-chirality Ls x Ls real matrices {'+': ..., '-': ...} of M_5, M_phi.

    On chirality + (spins 0,1) P_chi acts as S-, on chirality - as S+.
    """
    out = {}
    for chi, up in (("+", False), ("-", True)):
        S = shift_matrix(Ls, mf, up)
        alpha = b * (4 - M5) + 1
        beta = 1 - c * (4 - M5)
        out[chi] = {
            "S": S,
            "M5": alpha * np.eye(Ls) - beta * S,
            "Mphi": b * np.eye(Ls) + c * S,
            "alpha": alpha,
            "beta": beta,
        }
    return out


def m5inv_closed_form(Ls, M5, mf, b, c, chi):
    """(alpha - beta S)^{-1} = sum_k q^k S^k / (alpha (1 + mf q^Ls)), q = beta/alpha."""
    blk = chiral_blocks(Ls, M5, mf, b, c)[chi]
    alpha, beta, S = blk["alpha"], blk["beta"], blk["S"]
    q = beta / alpha
    acc = np.zeros((Ls, Ls))
    Sk = np.eye(Ls)
    for k in range(Ls):
        acc += q**k * Sk
        Sk = Sk @ S
    return acc / (alpha * (1 + mf * q**Ls))


def embed_chiral(Ls, plus, minus):
    """(4Ls)x(4Ls) matrix on index 4s+spin from per-chirality Ls x Ls blocks."""
    M = np.zeros((4 * Ls, 4 * Ls), complex)
    for sp in range(4):
        blk = plus if sp < 2 else minus
        for s in range(Ls):
            for t in range(Ls):
                M[4 * s + sp, 4 * t + sp] = blk[s, t]
    return M


# ----------------------------------------------------------------- dense matrices
def dense_of(apply, shape, dtype=np.complex128):
    """Dense matrix of a linear map by applying it to unit vectors."""
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype)
        e[j] = 1
        cols.append(np.asarray(apply(e.reshape(shape))).ravel())
    return np.stack(cols, axis=1)


def rand_c(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def momenta(L, tbc=-1):
    """All lattice momenta (antiperiodic in t when tbc = -1)."""
    ranges = []
    for mu, Lm in enumerate(L):
        shift = 0.5 if (mu == 3 and tbc < 0) else 0.0
        ranges.append([2 * np.pi * (n + shift) / Lm for n in range(Lm)])
    return [np.array(p) for p in itertools.product(*ranges)]
