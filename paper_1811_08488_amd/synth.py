"""Seeded synthetic inputs: SU(3) gauge fields and Gaussian sources.

This module only draws inputs.  It holds none of the solver's or the Dirac
operator's arithmetic, and both the GPU library's tests/benchmark and the CPU
oracle consume exactly the arrays it returns, so no random-number generator has
to be reproduced on either side.

Recipe (the paper measures on thermalised 2+1-flavour Moebius ensembles that
are not available, Sec. 3; these fields stand in for them):

* links   U_mu(x) = reunitarise(exp(i eps sum_a xi_a lambda_a / 2)),
          xi_a ~ N(0, 1) drawn in the order [lex][mu][a] from
          ``numpy.random.default_rng(seed)`` (PCG64), lambda_a the Gell-Mann
          matrices (tr lambda_a lambda_b = 2 delta_ab).  Reunitarisation is
          Gram-Schmidt of rows 0 and 1 with row 2 = conj(row0 x row1), so
          every link is exactly in SU(3) to rounding.
* eps     either given (0.3 for the small Shamir lattice) or tuned by bisection
          so that the average plaquette of a reference 8^4 field is 0.6, the
          value of a thermalised field.
* source  complex Gaussian 5D spinor on both parities,
          [rhs][lex][s][spin][colour], Re and Im ~ N(0, 1/2) so E|z|^2 = 1.
"""
from __future__ import annotations

import functools

import numpy as np
import torch


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape [8, 3, 3]."""
    l = np.zeros((8, 3, 3), np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def reunitarise(U: np.ndarray) -> np.ndarray:
    """Project [..., 3, 3] matrices onto SU(3) by Gram-Schmidt on rows 0, 1."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _expi(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) of Hermitian [..., 3, 3] matrices (torch CPU matrix_exp)."""
    t = torch.from_numpy(np.ascontiguousarray(1j * eps * H))
    return torch.linalg.matrix_exp(t).numpy()


def random_su3(n: int, eps: float, rng: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """n links exp(i eps xi.lambda/2), reunitarised; xi drawn [n][8] from rng."""
    lam = gell_mann()
    out = np.empty((n, 3, 3), np.complex128)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        xi = rng.standard_normal((m, 8))
        H = np.einsum("na,aij->nij", xi, lam) * 0.5
        out[s : s + m] = reunitarise(_expi(H, eps))
    return out


def gauge_field(L, eps: float, seed: int) -> np.ndarray:
    """U[lex][mu][row][col] complex128, lex = x + Lx(y + Ly(z + Lz t))."""
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    return random_su3(V * 4, eps, rng).reshape(V, 4, 3, 3)


def plaquette(U: np.ndarray, L) -> float:
    """(1/(18 V)) sum_x sum_{mu<nu} Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+."""
    Lx, Ly, Lz, Lt = L
    G = U.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu = G[..., mu, :, :]
            Unu = G[..., nu, :, :]
            Unu_xmu = np.roll(Unu, -1, axis=axis[mu])
            Umu_xnu = np.roll(Umu, -1, axis=axis[nu])
            t = Umu @ Unu_xmu @ np.conj(np.swapaxes(Umu_xnu, -1, -2)) @ np.conj(np.swapaxes(Unu, -1, -2))
            acc += np.real(np.trace(t, axis1=-2, axis2=-1)).sum()
    return acc / (18.0 * np.prod(L))


@functools.lru_cache(maxsize=None)
def tuned_eps(target: float = 0.6, seed: int = 777, L=(8, 8, 8, 8)) -> float:
    """Width eps for which a seeded reference field has average plaquette `target`."""
    lo, hi = 0.05, 1.5  # plaquette decreases monotonically with eps on this range
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if plaquette(gauge_field(L, mid, seed), L) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def source(L, Ls: int, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian phi[rhs][lex][s][spin][colour], E|z|^2 = 1."""
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    re_im = rng.standard_normal((nrhs, V, Ls, 4, 3, 2)) * np.sqrt(0.5)
    return re_im[..., 0] + 1j * re_im[..., 1]


def source_cb_chunks(L, Ls: int, nrhs: int, seed: int, sites_per_chunk: int = 1 << 20):
    """The same numbers as source(), drawn in order without holding the whole
    field: yields (rhs, cb0, even, odd) with even/odd = phi at the cb sites
    [cb0, cb0 + n) of each parity, [n][Ls][4][3].  Chunks cover whole pairs of
    lex sites (Lx even), so each holds the same cb range of both parities."""
    V = int(np.prod(L))
    Lx = L[0]
    step = max(2 * Lx, (sites_per_chunk // (2 * Lx)) * 2 * Lx)
    rng = np.random.default_rng(seed)
    for r in range(nrhs):
        for a in range(0, V, step):
            b = min(V, a + step)
            re_im = rng.standard_normal((b - a, Ls, 4, 3, 2)) * np.sqrt(0.5)
            phi = re_im[..., 0] + 1j * re_im[..., 1]
            lex = np.arange(a, b)
            x = lex % Lx
            rest = lex // Lx
            y = rest % L[1]
            rest //= L[1]
            z = rest % L[2]
            t = rest // L[2]
            par = (x + y + z + t) & 1
            yield r, a // 2, phi[par == 0], phi[par == 1]


def cb_field(L, Ls: int, nrhs: int, seed: int) -> np.ndarray:
    """Gaussian field on one parity, [rhs][V/2][Ls][4][3] (for operator tests)."""
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    re_im = rng.standard_normal((nrhs, V // 2, Ls, 4, 3, 2)) * np.sqrt(0.5)
    return re_im[..., 0] + 1j * re_im[..., 1]


def gauge_transform(L, seed: int) -> np.ndarray:
    """Random site-dependent SU(3) matrices g[lex] (wide distribution)."""
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    return random_su3(V, 2.0, rng)
