"""ctypes binding of the C ABI in ``include/mspcg.h`` (libmspcg.so, HIP for gfx950).

Argument marshalling only: every operator and solver step runs in the HIP
library.  PyTorch provides device memory and streams.  Loading fails loudly
when the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmspcg.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
OK, NOT_CONVERGED, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENONFINITE = 0, 1, -1, -2, -3, -4, -5
MAX_LS, MAX_NRHS = 32, 16

EXPORTED = [
    "mspcg_create", "mspcg_destroy", "dslash_eo", "m5inv", "mdagm", "local_block_cg", "cg_solve", "mspcg_solve",
    "dwf_prepare_rhs", "dwf_reconstruct", "mspcg_debug_site_maps", "mspcg_debug_block_sites", "mspcg_convert",
    "mspcg_block_apply", "mspcg_debug_block_hop", "mdagm_noalloc", "mspcg_last_error",
]
# MSPCG_NOALLOC_SCRATCH_BYTES: scratch of mdagm_noalloc per GPU
NOALLOC_SCRATCH_BYTES = 64 << 20


class Dwf(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("Ls", ctypes.c_int), ("M5", ctypes.c_double), ("mf", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double), ("t_bc", ctypes.c_int)]


class CField(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("norm", ctypes.c_void_p), ("prec", ctypes.c_int),
                ("nrhs", ctypes.c_int), ("parity", ctypes.c_int)]


class Precond(ctypes.Structure):
    _fields_ = [("nblk", ctypes.c_int * 4), ("n_inner", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("no_snake", ctypes.c_int), ("inner_tol", ctypes.c_double), ("n_sweeps", ctypes.c_int)]


class Solver(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("reliable_interval", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("timing", ctypes.c_int), ("flexible_beta", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_longlong),
                ("true_rel_resid", ctypes.POINTER(ctypes.c_double)), ("seconds", ctypes.c_double),
                ("t_outer_op", ctypes.c_double), ("t_precond", ctypes.c_double), ("t_blas", ctypes.c_double)]


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run paper_1811_08488_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, I = ctypes.c_void_p, ctypes.c_int
        FP = ctypes.POINTER(CField)
        sigs = {
            "mspcg_create": [ctypes.POINTER(P), ctypes.POINTER(Dwf), P, P],
            "mspcg_destroy": [P],
            "dslash_eo": [P, FP, FP, I, P],
            "m5inv": [P, FP, FP, I, P],
            "mdagm": [P, FP, FP, P],
            "local_block_cg": [P, FP, FP, ctypes.POINTER(Precond), P],
            "cg_solve": [P, FP, FP, ctypes.POINTER(Solver), ctypes.POINTER(Stats)],
            "mspcg_solve": [P, FP, FP, ctypes.POINTER(Solver), ctypes.POINTER(Precond), ctypes.POINTER(Stats)],
            "dwf_prepare_rhs": [P, FP, FP, FP, P],
            "dwf_reconstruct": [P, FP, FP, FP, P],
            "mspcg_debug_site_maps": [P, I, P, P],
            "mspcg_debug_block_sites": [P, P, I, P, P, P, P],
            "mspcg_convert": [P, FP, FP, P],
            "mspcg_block_apply": [P, FP, FP, ctypes.POINTER(Precond), P],
            "mspcg_debug_block_hop": [P, ctypes.POINTER(Precond), I, I, I, P, P],
            "mdagm_noalloc": [P, FP, FP, P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.mspcg_last_error.argtypes = []
        L.mspcg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class MspcgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise MspcgError(rc, lib().mspcg_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


@dataclass
class Action:
    L: tuple
    Ls: int
    M5: float = 1.8
    mf: float = 0.01
    b: float = 1.0
    c: float = 0.0
    t_bc: int = -1

    @property
    def V(self):
        return int(np.prod(self.L))


def to_device_layout(a: np.ndarray) -> np.ndarray:
    """complex128 [nrhs, sites, Ls, 4, 3] -> flat float64 in the F64 field layout
    [rhs][site][chunk][s][2 reals] (12 chunks of 2 reals per 5D site)."""
    nrhs, ns, Ls = a.shape[:3]
    r = a.view(np.float64).reshape(nrhs, ns, Ls, 12, 2)
    return np.ascontiguousarray(r.transpose(0, 1, 3, 2, 4)).reshape(-1)


def from_device_layout(flat: np.ndarray, nrhs: int, ns: int, Ls: int) -> np.ndarray:
    r = flat.reshape(nrhs, ns, 12, Ls, 2).transpose(0, 1, 3, 2, 4)
    return np.ascontiguousarray(r).view(np.complex128).reshape(nrhs, ns, Ls, 4, 3)


class Field:
    """One parity of a 5D field in device memory (layout of include/mspcg.h) plus the F16/BF16 norms."""

    def __init__(self, data, norm, prec, nrhs, parity):
        self.data, self.norm, self.prec, self.nrhs, self.parity = data, norm, prec, nrhs, parity

    def c(self):
        return CField(self.data.data_ptr(), self.norm.data_ptr() if self.norm is not None else None,
                      self.prec, self.nrhs, self.parity)


def _torch():
    import torch

    return torch


def new_field(A: Action, prec: int, nrhs: int, parity: int, device="cuda") -> Field:
    torch = _torch()
    n5 = nrhs * (A.V // 2) * A.Ls
    dt = {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[prec]
    data = torch.zeros(n5 * 24, dtype=dt, device=device)
    norm = torch.zeros(n5, dtype=torch.float32, device=device) if prec in (F16, BF16) else None
    return Field(data, norm, prec, nrhs, parity)


class Handle:
    """An MSPCG handle for one lattice, action and gauge field (FP64 [V,4,3,3] complex)."""

    def __init__(self, A: Action, gauge, stream=None):
        torch = _torch()
        self.A = A
        g = np.ascontiguousarray(gauge, dtype=np.complex128).view(np.float64)
        self._gauge = torch.from_numpy(g.reshape(-1)).to("cuda")
        d = Dwf((ctypes.c_int * 4)(*A.L), A.Ls, A.M5, A.mf, A.b, A.c, A.t_bc)
        h = ctypes.c_void_p()
        _check(lib().mspcg_create(ctypes.byref(h), ctypes.byref(d), ctypes.c_void_p(self._gauge.data_ptr()),
                                  _stream(stream)))
        self.h = h
        del self._gauge

    def close(self):
        if getattr(self, "h", None):
            lib().mspcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------- fields
    def field(self, prec, nrhs, parity) -> Field:
        return new_field(self.A, prec, nrhs, parity)

    def upload(self, arr, parity, prec=F64) -> Field:
        """complex128 [nrhs, V/2, Ls, 4, 3] (or without nrhs) -> device field of `prec`."""
        torch = _torch()
        a = np.ascontiguousarray(arr, dtype=np.complex128)
        if a.ndim == 4:
            a = a[None]
        nrhs = a.shape[0]
        f64 = Field(torch.from_numpy(to_device_layout(a)).to("cuda"), None, F64, nrhs, parity)
        if prec == F64:
            return f64
        out = self.field(prec, nrhs, parity)
        self.convert(out, f64)
        return out

    def download(self, f: Field) -> np.ndarray:
        """device field -> complex128 [nrhs, V/2, Ls, 4, 3]."""
        torch = _torch()
        if f.prec != F64:
            t = self.field(F64, f.nrhs, f.parity)
            self.convert(t, f)
            f = t
        torch.cuda.synchronize()
        return from_device_layout(f.data.cpu().numpy(), f.nrhs, self.A.V // 2, self.A.Ls)

    def write_sites(self, f: Field, cb, values):
        """Write complex128 [nrhs, n, Ls, 4, 3] into the listed cb sites of an F64 field."""
        torch = _torch()
        if f.prec != F64:
            raise ValueError("write_sites needs an F64 field")
        cb = np.asarray(cb, dtype=np.int64)
        v = to_device_layout(np.ascontiguousarray(values, dtype=np.complex128)).reshape(
            f.nrhs, len(cb), 12, self.A.Ls, 2)
        view = f.data.view(f.nrhs, self.A.V // 2, 12, self.A.Ls, 2)
        view[:, torch.from_numpy(cb).to(f.data.device)] = torch.from_numpy(v).to(f.data.device)

    def read_sites(self, f: Field, cb) -> np.ndarray:
        """The listed cb sites of a field as complex128 [nrhs, n, Ls, 4, 3]."""
        torch = _torch()
        if f.prec != F64:
            t = self.field(F64, f.nrhs, f.parity)
            self.convert(t, f)
            f = t
        cb = np.asarray(cb, dtype=np.int64)
        view = f.data.view(f.nrhs, self.A.V // 2, 12, self.A.Ls, 2)
        got = view[:, torch.from_numpy(cb).to(f.data.device)].cpu().numpy()
        return from_device_layout(got.reshape(-1), f.nrhs, len(cb), self.A.Ls)

    # -------------------------------------------------------- operators
    def convert(self, out: Field, inp: Field, stream=None):
        _check(lib().mspcg_convert(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), _stream(stream)))

    def dslash_eo(self, out: Field, inp: Field, dagger=0, stream=None):
        _check(lib().dslash_eo(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), int(dagger), _stream(stream)))

    def m5inv(self, out: Field, inp: Field, dagger=0, stream=None):
        _check(lib().m5inv(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), int(dagger), _stream(stream)))

    def mdagm(self, out: Field, inp: Field, stream=None):
        _check(lib().mdagm(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), _stream(stream)))

    def mdagm_noalloc(self, out: Field, inp: Field, stream=None):
        _check(lib().mdagm_noalloc(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), _stream(stream)))

    def block_apply(self, out: Field, inp: Field, nblk, prec=F64, stream=None, no_snake=0):
        pc = Precond((ctypes.c_int * 4)(*nblk), 0, int(prec), int(no_snake), 0.0, 1)
        _check(lib().mspcg_block_apply(self.h, ctypes.byref(out.c()), ctypes.byref(inp.c()), ctypes.byref(pc),
                                       _stream(stream)))

    def block_hop(self, nblk, prec, nrhs, hop, reps=1, stream=None, no_snake=0):
        """Launch block hop 1..4 of the inner iteration `reps` times; returns the 4D sites of its
        (input, output) domains summed over blocks."""
        pc = Precond((ctypes.c_int * 4)(*nblk), 0, int(prec), int(no_snake), 0.0, 1)
        n = (ctypes.c_longlong * 2)()
        _check(lib().mspcg_debug_block_hop(self.h, ctypes.byref(pc), int(nrhs), int(hop), int(reps), n,
                                           _stream(stream)))
        return int(n[0]), int(n[1])

    def local_block_cg(self, z: Field, r: Field, nblk, n_inner, inner_prec=F32, stream=None, no_snake=0,
                       inner_tol=0.0, n_sweeps=1):
        pc = Precond((ctypes.c_int * 4)(*nblk), int(n_inner), int(inner_prec), int(no_snake), float(inner_tol),
                     int(n_sweeps))
        _check(lib().local_block_cg(self.h, ctypes.byref(z.c()), ctypes.byref(r.c()), ctypes.byref(pc),
                                    _stream(stream)))

    def prepare_rhs(self, b: Field, phi_e: Field, phi_o: Field, stream=None):
        _check(lib().dwf_prepare_rhs(self.h, ctypes.byref(b.c()), ctypes.byref(phi_e.c()), ctypes.byref(phi_o.c()),
                                     _stream(stream)))

    def reconstruct(self, psi_o: Field, psi_e: Field, phi_o: Field, stream=None):
        _check(lib().dwf_reconstruct(self.h, ctypes.byref(psi_o.c()), ctypes.byref(psi_e.c()),
                                     ctypes.byref(phi_o.c()), _stream(stream)))

    # -------------------------------------------------------- solvers
    def _solve(self, x: Field, b: Field, tol, max_iter, reliable, precond, use_graph=1, timing=0, flexible_beta=0):
        resid = (ctypes.c_double * b.nrhs)()
        st = Stats(0, 0, ctypes.cast(resid, ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0.0)
        s = Solver(float(tol), int(max_iter), int(reliable), int(use_graph), int(timing), int(flexible_beta))
        if precond is None:
            rc = lib().cg_solve(self.h, ctypes.byref(x.c()), ctypes.byref(b.c()), ctypes.byref(s), ctypes.byref(st))
        else:
            nblk, k, prec, no_snake, inner_tol, n_sweeps = precond
            pc = Precond((ctypes.c_int * 4)(*nblk), int(k), int(prec), int(no_snake), float(inner_tol),
                         int(n_sweeps))
            rc = lib().mspcg_solve(self.h, ctypes.byref(x.c()), ctypes.byref(b.c()), ctypes.byref(s),
                                   ctypes.byref(pc), ctypes.byref(st))
        _check(rc, allow=(OK, NOT_CONVERGED))
        return {"status": rc, "outer_iters": st.outer_iters, "inner_iters": st.inner_iters,
                "true_rel_resid": list(resid), "seconds": st.seconds, "t_outer_op": st.t_outer_op,
                "t_precond": st.t_precond, "t_blas": st.t_blas}

    def cg_solve(self, x: Field, b: Field, tol=1e-10, max_iter=10000, reliable=50, timing=0):
        return self._solve(x, b, tol, max_iter, reliable, None, timing=timing)

    def mspcg_solve(self, x: Field, b: Field, nblk, n_inner, inner_prec=F32, tol=1e-10, max_iter=10000,
                    reliable=50, use_graph=1, no_snake=0, inner_tol=0.0, n_sweeps=1, timing=0, flexible_beta=0):
        return self._solve(x, b, tol, max_iter, reliable,
                           (nblk, n_inner, inner_prec, no_snake, inner_tol, n_sweeps), use_graph, timing,
                           flexible_beta)

    # -------------------------------------------------------- debug exports
    def site_maps(self, parity):
        Vh = self.A.V // 2
        lex = np.zeros(Vh, np.int32)
        nbr = np.zeros((Vh, 4, 2), np.int32)
        _check(lib().mspcg_debug_site_maps(self.h, int(parity), lex.ctypes.data_as(ctypes.c_void_p),
                                           nbr.ctypes.data_as(ctypes.c_void_p)))
        return lex, nbr

    def block_sites(self, nblk, block):
        counts = np.zeros(3, np.int32)
        nb = (ctypes.c_int * 4)(*nblk)
        _check(lib().mspcg_debug_block_sites(self.h, nb, int(block), counts.ctypes.data_as(ctypes.c_void_p),
                                             None, None, None))
        be, o1, e2 = (np.zeros(int(c), np.int32) for c in counts)
        _check(lib().mspcg_debug_block_sites(self.h, nb, int(block), counts.ctypes.data_as(ctypes.c_void_p),
                                             be.ctypes.data_as(ctypes.c_void_p), o1.ctypes.data_as(ctypes.c_void_p),
                                             e2.ctypes.data_as(ctypes.c_void_p)))
        return be, o1, e2
