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
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


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
