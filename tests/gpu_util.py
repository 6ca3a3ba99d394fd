"""Shared set-up for the GPU parity tests: the same seeded host arrays go to the
HIP library (through the C ABI) and to the FP64 CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import mspcg as M
from paper_1811_08488_amd import synth

MOBIUS = dict(M5=1.8, b=1.5, c=0.5)
SHAMIR = dict(M5=1.8, b=1.0, c=0.0)

# Per-application tolerances (relative 2-norm of the difference).
TOL = {M.F64: 1e-13, M.F32: 1e-6, M.F16: 5e-3, M.BF16: 5e-3}
PRECS = [M.F64, M.F32, M.F16, M.BF16]
PNAME = {M.F64: "f64", M.F32: "f32", M.F16: "f16", M.BF16: "bf16"}


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    """Relative 2-norm of the difference over the whole field."""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def site_err(got, want, floor=1e-3):
    """Largest element-wise error measured against the norm of its own 5D site:
    max over (rhs, site, s, spin, colour) of |got - want| / ||want_site||, a
    5D site being the 12 complex values of one (rhs, cb, s).  Sites whose norm
    is below `floor` times the field's RMS site norm are measured against that
    floor.  A single wrong spin-colour component anywhere fails it, unlike a
    norm over the whole field."""
    g = np.asarray(got).reshape(-1, 12)
    w = np.asarray(want).reshape(-1, 12)
    n = np.linalg.norm(w, axis=1)
    ref = np.maximum(n, floor * np.sqrt(np.mean(n * n)))
    if not np.all(ref > 0):
        return float(np.max(np.abs(g - w)))
    return float(np.max(np.abs(g - w) / ref[:, None]))


# Element-wise tolerances against the site norm, per application (one hop, one
# M_5^-1): the stored output rounds each real to u * n with n <= ||site|| (u the
# unit roundoff: FP32 2^-24, FP16 2^-11, BF16 2^-9), and the links stored in
# the same type add about u per product; the F16 hop also rounds its projected
# half spinor (2^-11).  Both are compared with the oracle applied to the
# rounded input the GPU received.
SITE_TOL = {M.F64: 1e-13, M.F32: 1e-6, M.F16: 5e-3, M.BF16: 5e-3}


def rounded(h, x, parity, prec):
    """The values a field of `prec` holds after an upload of x (what the kernels read)."""
    if prec == M.F64:
        return np.asarray(x)
    return h.download(h.upload(x, parity, prec))


class Setup:
    def __init__(self, L, Ls, kind="mobius", mf=0.05, eps=0.45, seed=1):
        prm = MOBIUS if kind == "mobius" else SHAMIR
        self.oa = O.Action(tuple(L), Ls, mf=mf, **prm)
        self.ga = M.Action(tuple(L), Ls, mf=mf, t_bc=-1, **prm)
        self.U = synth.gauge_field(L, eps, seed)
        self.h = M.Handle(self.ga, self.U)
        self.L, self.Ls = tuple(L), Ls
        self.Vh = int(np.prod(L)) // 2

    def rand(self, nrhs, seed):
        return synth.cb_field(self.L, self.Ls, nrhs, seed)
