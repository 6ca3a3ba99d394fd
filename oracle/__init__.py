"""FP64 CPU oracle for MSPCG on the even-odd preconditioned Moebius DWF operator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
imports, links or calls it, and this package shares no code with the GPU
library: the two are independent implementations of the same definitions.

The arithmetic lives in ``dwf_oracle.cpp`` (plain C++17 + OpenMP, FP64,
lexicographic full-lattice fields); this module is a ctypes wrapper around it
with numpy arrays:

* gauge      ``complex128[V, 4, 3, 3]``      U[lex][mu][row][col]
* lex field  ``complex128[V, Ls, 4, 3]``     psi[lex][s][spin][colour]
* cb field   ``complex128[V//2, Ls, 4, 3]``  one parity, cb = lex >> 1

Function-by-function citations (sections of the paper) are in the C++ source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwf_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place (g++ -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    sig = {
        "oracle_site_maps": [_P, _I, _P, _P],
        "oracle_block_of_site": [_P, _P, _P],
        "oracle_op5_matrix": [_I, _P, _I, _P],
        "oracle_hop_full": [_P, _I, _P, _P, _P, _P, _I],
        "oracle_D_full": [_P, _I, _P, _P, _P, _P],
        "oracle_dslash_eo": [_P, _I, _P, _P, _P, _P, _I, _I],
        "oracle_op5": [_P, _I, _P, _P, _P, _I, _I],
        "oracle_dpc": [_P, _I, _P, _P, _P, _P, _I, _I],
        "oracle_mdagm": [_P, _I, _P, _P, _P, _P],
        "oracle_prepare_rhs": [_P, _I, _P, _P, _P, _P, _P],
        "oracle_reconstruct": [_P, _I, _P, _P, _P, _P, _P],
        "oracle_block_op": [_P, _I, _P, _P, _P, _P, _P, _I, _I],
        "oracle_local_block_cg": [_P, _I, _P, _P, _P, _P, _P, _I, _I, _D, _I],
        "oracle_solve": [_P, _I, _P, _P, _P, _P, _P, _I, _I, _D, _I, _I, _P, _P, _I, _D, _I, _I],
        "oracle_num_threads": [],
        "oracle_set_num_threads": [_I],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = None if name == "oracle_set_num_threads" else _I


# Operator selectors of oracle_op5 / op5_matrix
M5, M5_DAG, M5INV, M5INV_DAG, MPHI, MPHI_DAG, PCHI = range(7)


@dataclass(frozen=True)
class Action:
    """Lattice and Moebius-DWF parameters (Shamir: b=1, c=0)."""

    L: tuple  # (Lx, Ly, Lz, Lt)
    Ls: int
    M5: float = 1.8
    mf: float = 0.01
    b: float = 1.0
    c: float = 0.0
    tbc: float = -1.0  # time boundary factor (-1: antiperiodic)

    @property
    def V(self) -> int:
        return int(np.prod(self.L))

    def cL(self):
        return (ctypes.c_int * 4)(*self.L)

    def cp(self):
        return (ctypes.c_double * 5)(self.M5, self.mf, self.b, self.c, self.tbc)


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name}: invalid arguments (rc={rc})")


def _cb_shape(A: Action):
    return (A.V // 2, A.Ls, 4, 3)


def _lex_shape(A: Action):
    return (A.V, A.Ls, 4, 3)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def site_maps(L, parity: int):
    """(lex_of_cb[V/2], nbr[V/2, 4, 2]) for one parity; nbr[..., 0] = x+mu, 1 = x-mu."""
    V = int(np.prod(L))
    lex = np.zeros(V // 2, np.int32)
    nbr = np.zeros((V // 2, 4, 2), np.int32)
    _check(lib().oracle_site_maps((ctypes.c_int * 4)(*L), parity, _ptr(lex), _ptr(nbr)), "site_maps")
    return lex, nbr


def block_of_site(L, nblk):
    V = int(np.prod(L))
    out = np.zeros(V, np.int32)
    _check(
        lib().oracle_block_of_site((ctypes.c_int * 4)(*L), (ctypes.c_int * 4)(*nblk), _ptr(out)),
        "block_of_site",
    )
    return out


def op5_matrix(A: Action, which: int) -> np.ndarray:
    n = 4 * A.Ls
    m = np.zeros((n, n), np.complex128)
    _check(lib().oracle_op5_matrix(A.Ls, A.cp(), which, _ptr(m)), "op5_matrix")
    return m


def hop_full(A: Action, U, psi, sign: int = +1) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_lex_shape(A), np.complex128)
    _check(lib().oracle_hop_full(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi), sign), "hop_full")
    return out


def D_full(A: Action, U, psi) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_lex_shape(A), np.complex128)
    _check(lib().oracle_D_full(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi)), "D_full")
    return out


def dslash_eo(A: Action, U, psi, out_parity: int, dagger: int = 0) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_cb_shape(A), np.complex128)
    _check(
        lib().oracle_dslash_eo(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi), out_parity, dagger),
        "dslash_eo",
    )
    return out


def op5(A: Action, psi, which: int, parity: int = 0) -> np.ndarray:
    psi = _c128(psi)
    out = np.zeros(_cb_shape(A), np.complex128)
    _check(lib().oracle_op5(A.cL(), A.Ls, A.cp(), _ptr(out), _ptr(psi), parity, which), "op5")
    return out


def dpc(A: Action, U, psi, parity: int = 0, dagger: int = 0) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_cb_shape(A), np.complex128)
    _check(lib().oracle_dpc(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi), parity, dagger), "dpc")
    return out


def mdagm(A: Action, U, psi) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_cb_shape(A), np.complex128)
    _check(lib().oracle_mdagm(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi)), "mdagm")
    return out


def prepare_rhs(A: Action, U, phi_lex):
    """(b, phihat_e): b = D_PC^+ phihat_e, phihat_e = phi_e - M4_eo M5^-1 phi_o."""
    U, phi = _c128(U), _c128(phi_lex)
    b = np.zeros(_cb_shape(A), np.complex128)
    ph = np.zeros(_cb_shape(A), np.complex128)
    _check(lib().oracle_prepare_rhs(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(b), _ptr(ph), _ptr(phi)), "prepare_rhs")
    return b, ph


def reconstruct(A: Action, U, psi_e, phi_lex) -> np.ndarray:
    U, pe, phi = _c128(U), _c128(psi_e), _c128(phi_lex)
    out = np.zeros(_lex_shape(A), np.complex128)
    _check(lib().oracle_reconstruct(A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(pe), _ptr(phi)), "reconstruct")
    return out


def block_op(A: Action, U, psi, nblk, block: int, truncated: bool = False) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.zeros(_cb_shape(A), np.complex128)
    _check(
        lib().oracle_block_op(
            A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(out), _ptr(psi), (ctypes.c_int * 4)(*nblk), block, int(truncated)
        ),
        "block_op",
    )
    return out


def local_block_cg(A: Action, U, r, nblk, k: int, truncated: bool = False, inner_tol: float = 0.0,
                   sweeps: int = 1) -> np.ndarray:
    """z = sum_s P_s CG_k(A_s, P_s r) (Sec. 2.4).  inner_tol > 0: each block stops after the first
    iteration with |r_s| <= inner_tol |P_s r| (the precision-based stopping Sec. 3 sets aside).
    sweeps > 1: further multisplitting sweeps z <- z + M (r - A z) (Sec. 2.1)."""
    U, r = _c128(U), _c128(r)
    z = np.zeros(_cb_shape(A), np.complex128)
    _check(
        lib().oracle_local_block_cg(
            A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(z), _ptr(r), (ctypes.c_int * 4)(*nblk), k, int(truncated),
            float(inner_tol), int(sweeps),
        ),
        "local_block_cg",
    )
    return z


@dataclass
class SolveStats:
    iters: int
    true_rel_resid: float
    converged: bool
    history: np.ndarray


def solve(A: Action, U, b, x0=None, nblk=None, k: int = 0, truncated: bool = False, tol: float = 1e-10,
          maxiter: int = 10000, reliable: int = 50, hist_len: int = 0, inner_tol: float = 0.0, sweeps: int = 1,
          flexible: bool = False):
    """Algorithm 1 on D_PC^+ D_PC x = b.  nblk=None: plain CG; else MSPCG with k inner CG iterations.
    flexible: the Polak-Ribiere beta <z', r' - r> / <z, r> instead of the printed Fletcher-Reeves one."""
    U, b = _c128(U), _c128(b)
    x = np.zeros(_cb_shape(A), np.complex128) if x0 is None else _c128(x0).copy()
    st = np.zeros(3, np.float64)
    hist = np.zeros(max(hist_len, 1), np.float64)
    nb = None if nblk is None else (ctypes.c_int * 4)(*nblk)
    _check(
        lib().oracle_solve(
            A.cL(), A.Ls, A.cp(), _ptr(U), _ptr(x), _ptr(b), nb, k, int(truncated), tol, maxiter, reliable,
            _ptr(st), _ptr(hist), hist_len, float(inner_tol), int(sweeps), int(bool(flexible)),
        ),
        "solve",
    )
    return x, SolveStats(int(st[0]), float(st[1]), bool(st[2]), hist[: max(0, min(hist_len, int(st[0]) + 1))])
