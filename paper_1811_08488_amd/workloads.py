"""The five synthetic workloads (lattice, action, solver and preconditioner settings).

Pure data: no arithmetic.  Seeds: gauge 1000+i, source 2000+i for workload i.
Where a workload leaves a value open the choice is marked ``assumed``.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    L: tuple            # (Lx, Ly, Lz, Lt)
    Ls: int
    M5: float
    mf: float
    b: float
    c: float
    nrhs: int
    eps: float | None   # link width; None = tuned for plaquette 0.6
    nblk: tuple | None  # blocks per dimension (None: plain CG only)
    n_inner: int
    inner_prec: str     # "f32", "f16", "bf16"
    tol: float = 1e-10
    reliable: int = 50
    gauge_seed: int = 0
    source_seed: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        v = 1
        for x in self.L:
            v *= x
        return v


WORKLOADS = {
    # Shamir DWF on 4^4 x 8, plain FP64 CG.
    "shamir_4x4x4x4_ls8": Workload(
        "shamir_4x4x4x4_ls8", (4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0, 1, 0.3, None, 0, "f32",
        gauge_seed=1000, source_seed=2000),
    # Moebius on 16^3x32 x 16, 2^4 blocks of 8^3x16, 6 inner FP32 iterations.
    "mobius_16x16x16x32_ls16": Workload(
        "mobius_16x16x16x32_ls16", (16, 16, 16, 32), 16, 1.8, 0.01, 1.5, 0.5, 1, None, (2, 2, 2, 2), 6, "f32",
        gauge_seed=1001, source_seed=2001, notes={"reliable": "assumed 50"}),
    # Moebius on 24^3x64 x 24, light mass, 2x2x2x4 blocks of 12^3x16, 8 inner FP16.
    "mobius_24x24x24x64_ls24": Workload(
        "mobius_24x24x24x64_ls24", (24, 24, 24, 64), 24, 1.8, 0.00107, 1.5, 0.5, 1, None, (2, 2, 2, 4), 8, "f16",
        gauge_seed=1002, source_seed=2002),
    # 8 right-hand sides, uneven 3x3x3x4 blocks (11/11/10 x 16), BF16 and FP16 inner.
    "mobius_32x32x32x64_ls12_rhs8": Workload(
        "mobius_32x32x32x64_ls12_rhs8", (32, 32, 32, 64), 12, 1.8, 0.005, 1.5, 0.5, 8, None, (3, 3, 3, 4), 6, "bf16",
        gauge_seed=1003, source_seed=2003, notes={"M5": "assumed 1.8", "n_inner": "assumed 6"}),
    # Large single-GPU volume 48^3x96 x 12, 4^4 blocks of 12^3x24, 6 inner FP16.
    "mobius_48x48x48x96_ls12": Workload(
        "mobius_48x48x48x96_ls12", (48, 48, 48, 96), 12, 1.8, 0.00078, 1.5, 0.5, 1, None, (4, 4, 4, 4), 6, "f16",
        gauge_seed=1004, source_seed=2004, notes={"reliable": "assumed 50"}),
}

ORDER = list(WORKLOADS)
