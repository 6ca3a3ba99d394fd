"""Host logic of bench.py (CPU): the one-GPU guard, the algorithmic byte
counts behind the roofline figures, and the reading of the committed counter
summaries."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1811_08488_amd import mspcg as M  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_dslash_bytes_per_site():
    # in + out spinor of one 5D site (with the F16/BF16 norm) and the 8 x 18
    # link reals of its 4D site shared by the Ls sites: 456 / 228 / 122 bytes
    # at Ls = 16, one right-hand side
    assert bench.dslash_bytes_per_site(M.F64, 16, 1) == 2 * 24 * 8 + 144 * 8 / 16 == 456
    assert bench.dslash_bytes_per_site(M.F32, 16, 1) == 228
    assert bench.dslash_bytes_per_site(M.F16, 16, 1) == 122
    assert bench.dslash_bytes_per_site(M.BF16, 16, 1) == 122
    # links amortised over the right-hand sides too
    assert bench.dslash_bytes_per_site(M.F64, 12, 8) == 2 * 192 + 1152 / 96


def halo_counts(L, block):
    """Even sites of a block, odd sites within one hop of it, even sites within
    two hops (periodic lattice L, block [0, block_mu) in every direction),
    by brute force over the lattice."""
    axes = [np.arange(n) for n in L]
    grid = np.meshgrid(*axes, indexing="ij")
    dist = np.zeros(tuple(L), dtype=np.int64)
    for x, n, b in zip(grid, L, block):
        below = (-x) % n           # distance up to the block's first coordinate 0
        above = (x - (b - 1)) % n  # distance down to its last coordinate b - 1
        dist += np.where(x < b, 0, np.minimum(below, above))
    parity = sum(grid) % 2
    be = int(np.sum((dist == 0) & (parity == 0)))
    o1 = int(np.sum((dist <= 1) & (parity == 1)))
    e2 = int(np.sum((dist <= 2) & (parity == 0)))
    return be, o1, e2


def test_block_hop_bytes_on_24x24x24x64():
    # 2 x 2 x 2 x 4 blocks of 12^3 x 16: the domains of one block, counted
    # here, times 32 blocks; hop 2 reads O1, writes E2 and reads the block's
    # own p (M_5 p), in FP16 with norms at Ls = 24
    be, o1, e2 = halo_counts((24, 24, 24, 64), (12, 12, 12, 16))
    assert (be, o1, e2) == (13824, 22464, 33120)
    nb = 32
    got = bench.block_hop_bytes(M.F16, 24, 1, nb * o1, nb * e2, nb * be)
    site5 = (24 * 2 + 4) * 24
    assert got == (nb * (o1 + e2 + be)) * site5 + nb * e2 * 144 * 2 == 3077111808


def test_measured_traffic_follows_the_kernel_sources(monkeypatch):
    w = "mobius_24x24x24x64_ls24"
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{w}.txt")
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    labels = [k[len("traffic_bytes_per_launch_"):] for k in kv if k.startswith("traffic_bytes_per_launch_")]
    assert "block_hop2_f16" in labels and "dslash_eo_f64" in labels
    # each figure is (FETCH_SIZE x read factor + WRITE_SIZE x write factor)
    # KiB (the factors are printed to 4 decimals)
    for lab in labels:
        want = (float(kv[f"fetch_kib_{lab}"]) * float(kv["read_factor"]) +
                float(kv[f"write_kib_{lab}"]) * float(kv["write_factor"])) * 1024
        assert abs(float(kv[f"traffic_bytes_per_launch_{lab}"]) - want) <= 1e-4 * want
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: kv["kernel_source_sha256"])
    for lab in labels:
        assert bench.measured_traffic(w, lab) == float(kv[f"traffic_bytes_per_launch_{lab}"])
    assert bench.measured_traffic(w, "no_such_kernel") is None
    assert bench.measured_traffic("no_such_workload", "block_hop2_f16") is None
    # kernels changed since the counters were taken: no figure
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(w, "block_hop2_f16") is None


@pytest.mark.parametrize("prec", [M.F64, M.F32, M.F16, M.BF16])
def test_block_hop_bytes_scale_with_the_domains(prec):
    w, n = bench.BYTES[prec]
    a = bench.block_hop_bytes(prec, 12, 2, 100, 200, 50)
    assert a == 350 * (24 * w + n) * 12 * 2 + 200 * 144 * w
