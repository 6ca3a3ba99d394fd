"""Pins of the oracle's block operator, fixed-k inner CG and Algorithm 1 (CPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_1811_08488_amd import synth
from tests import lattice_helpers as H

MOB = dict(M5=1.8, mf=0.1, b=1.5, c=0.5)


def block_mask(L, nblk, block, Ls):
    blk = O.block_of_site(L, nblk)
    m = H.full_to_cb(L, (blk == block).astype(float)[:, None, None, None] * np.ones((1, Ls, 4, 3)), 0)
    return m


def dense_block_op(A, U, nblk, block, truncated=False):
    """A_s restricted to the block's even sites, as a dense matrix on those coordinates."""
    m = block_mask(A.L, nblk, block, A.Ls).astype(bool)
    idx = np.nonzero(m.ravel())[0]

    def apply(v):
        full = np.zeros(m.size, complex)
        full[idx] = v.ravel()
        return O.block_op(A, U, full.reshape(m.shape), nblk, block, truncated).ravel()[idx]

    return H.dense_of(apply, (len(idx),)), idx, m


@pytest.fixture(scope="module")
def small():
    A = O.Action((4, 4, 4, 4), 4, **MOB)
    U = synth.gauge_field(A.L, 0.5, 71)
    return A, U


def test_block_op_hpd_and_local(small):
    A, U = small
    nblk = (2, 2, 2, 2)
    M, idx, m = dense_block_op(A, U, nblk, 6)
    assert np.abs(M - M.conj().T).max() < 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    rng = np.random.default_rng(6)
    v = H.rand_c(rng, m.shape)
    out = O.block_op(A, U, v, nblk, 6)
    assert np.all(out[~m] == 0)  # output restricted to the block
    # input outside the block does not matter
    assert np.array_equal(out, O.block_op(A, U, v * m, nblk, 6))


def test_block_equal_to_lattice_is_full_operator(small):
    A, U = small
    rng = np.random.default_rng(7)
    v = H.rand_c(rng, (A.V // 2, A.Ls, 4, 3))
    assert np.abs(O.block_op(A, U, v, (1, 1, 1, 1), 0) - O.mdagm(A, U, v)).max() == 0


def test_snake_terms_only_near_the_boundary():
    """A_s and the truncated operator differ only for sites near the block boundary."""
    A = O.Action((4, 4, 4, 16), 4, **MOB)
    U = synth.gauge_field(A.L, 0.5, 81)
    nblk = (1, 1, 1, 2)  # blocks t in [0, 8) and [8, 16); boundary only in t
    c = H.coords_of_lex(A.L)
    par = c.sum(1) % 2
    rng = np.random.default_rng(8)
    for t, deep in ((4, True), (0, False), (7, False)):
        sites = np.nonzero((c[:, 3] == t) & (par == 0))[0]
        full = np.zeros((A.V, A.Ls, 4, 3), complex)
        full[sites] = H.rand_c(rng, (len(sites), A.Ls, 4, 3))
        v = H.full_to_cb(A.L, full, 0)
        d = O.block_op(A, U, v, nblk, 0, False) - O.block_op(A, U, v, nblk, 0, True)
        scale = np.abs(O.block_op(A, U, v, nblk, 0, False)).max()
        if deep:
            assert np.abs(d).max() < 1e-14 * scale
        else:
            assert np.abs(d).max() > 1e-3 * scale


def test_inner_tol_zero_is_fixed_k(small):
    A, U = small
    r = H.rand_c(np.random.default_rng(31), (A.V // 2, A.Ls, 4, 3))
    for k in (1, 4):
        assert np.array_equal(O.local_block_cg(A, U, r, (2, 1, 1, 2), k),
                              O.local_block_cg(A, U, r, (2, 1, 1, 2), k, inner_tol=0.0))


def test_inner_tol_stops_each_block_at_its_first_crossing(small):
    """Precision-based stopping (Sec. 3, the alternative to a fixed k): every
    block's result equals fixed-k CG on that block with k the first iteration
    count whose residual |P_s r - A_s z_s| is at most tol |P_s r| (kmax if
    none), found by brute force over k with the fixed-k oracle."""
    A, U = small
    nblk, kmax, tol = (2, 1, 1, 2), 8, 0.045
    r = H.rand_c(np.random.default_rng(32), (A.V // 2, A.Ls, 4, 3))
    fixed = {k: O.local_block_cg(A, U, r, nblk, k) for k in range(1, kmax + 1)}
    got = O.local_block_cg(A, U, r, nblk, kmax, inner_tol=tol)
    stops = []
    for b in range(int(np.prod(nblk))):
        m = block_mask(A.L, nblk, b, A.Ls)
        rs = r * m
        kstar = kmax
        for k in range(1, kmax + 1):
            res = np.linalg.norm(rs - O.block_op(A, U, fixed[k] * m, nblk, b)) / np.linalg.norm(rs)
            assert abs(res - tol) > 1e-6 * tol  # no borderline decision
            if res <= tol:
                kstar = k
                break
        stops.append(kstar)
        want = fixed[kstar] * m
        assert np.linalg.norm(got * m - want) <= 1e-12 * np.linalg.norm(want), (b, kstar)
    # the criterion is reached, at different iterations in different blocks
    assert max(stops) < kmax and len(set(stops)) > 1, stops


def test_multisplit_sweeps_are_block_jacobi_steps():
    """Several multisplitting sweeps (Sec. 2.1) with exact block solves: s sweeps
    give sum_{j<s} (I - B A)^j B r with B = (+)_s A_s^{-1} the exact block inverse
    (dense matrices on 2^3x4 x Ls=4), and one sweep is the single-sweep
    preconditioner unchanged."""
    A = O.Action((2, 2, 2, 4), 4, **MOB)
    U = synth.gauge_field(A.L, 0.5, 91)
    nblk = (1, 1, 1, 2)
    shape = (A.V // 2, A.Ls, 4, 3)
    Ad = H.dense_of(lambda v: O.mdagm(A, U, v), shape)
    B = np.zeros_like(Ad)
    for b in range(2):
        Ms, idx, _ = dense_block_op(A, U, nblk, b)
        B[np.ix_(idx, idx)] = np.linalg.inv(Ms)
    r = H.rand_c(np.random.default_rng(33), shape)
    k = 200  # CG on each 384-dimensional block converges to rounding
    assert np.array_equal(O.local_block_cg(A, U, r, nblk, 5), O.local_block_cg(A, U, r, nblk, 5, sweeps=1))
    IBA = np.eye(len(Ad)) - B @ Ad
    for sweeps in (1, 2, 3):
        want = sum(np.linalg.matrix_power(IBA, j) for j in range(sweeps)) @ (B @ r.ravel())
        got = O.local_block_cg(A, U, r, nblk, k, sweeps=sweeps).ravel()
        assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want), sweeps


def test_inner_cg_k1_closed_form(small):
    A, U = small
    nblk = (2, 2, 2, 2)
    rng = np.random.default_rng(9)
    r = H.rand_c(rng, (A.V // 2, A.Ls, 4, 3))
    z = O.local_block_cg(A, U, r, nblk, 1)
    want = np.zeros_like(r)
    for s in range(16):
        rs = r * block_mask(A.L, nblk, s, A.Ls)
        Ars = O.block_op(A, U, rs, nblk, s)
        want += (np.vdot(rs, rs).real / np.vdot(rs, Ars).real) * rs
    assert np.abs(z - want).max() < 1e-13 * np.abs(want).max()


def test_inner_cg_krylov_minimiser_and_exact_termination(small):
    A, U = small
    nblk = (2, 2, 2, 2)
    s = 9
    M, idx, m = dense_block_op(A, U, nblk, s)
    rng = np.random.default_rng(10)
    r = H.rand_c(rng, (A.V // 2, A.Ls, 4, 3)) * m
    rs = r.ravel()[idx]
    for k in (2, 3, 5):
        z = O.local_block_cg(A, U, r, (2, 2, 2, 2), k).ravel()
        # every block runs its own CG; look at block s only
        zs = z[idx]
        # minimiser of the A-norm error over K_k(A_s, r_s): Galerkin on an orthonormal basis
        K = np.stack([np.linalg.matrix_power(M, j) @ rs for j in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        y = np.linalg.solve(Q.conj().T @ M @ Q, Q.conj().T @ rs)
        want = Q @ y
        assert np.abs(zs - want).max() < 1e-9 * np.abs(want).max()
    # many iterations: the block system is solved
    z = O.local_block_cg(A, U, r, nblk, 400).ravel()[idx]
    exact = np.linalg.solve(M, rs)
    assert np.abs(z - exact).max() < 1e-9 * np.abs(exact).max()


def test_inner_cg_scale_equivariance(small):
    A, U = small
    rng = np.random.default_rng(11)
    r = H.rand_c(rng, (A.V // 2, A.Ls, 4, 3))
    z1 = O.local_block_cg(A, U, r, (2, 2, 1, 2), 4)
    z2 = O.local_block_cg(A, U, 1e-7 * r, (2, 2, 1, 2), 4)
    assert np.abs(z2 - 1e-7 * z1).max() < 1e-13 * np.abs(z2).max()


def test_inner_cg_zero_residual_block_stays_zero(small):
    A, U = small
    nblk = (2, 2, 2, 2)
    rng = np.random.default_rng(12)
    r = H.rand_c(rng, (A.V // 2, A.Ls, 4, 3)) * block_mask(A.L, nblk, 3, A.Ls)
    z = O.local_block_cg(A, U, r, nblk, 3)
    assert np.all(z[block_mask(A.L, nblk, 3, A.Ls) == 0] == 0)
    assert np.isfinite(z).all()


def test_cg_and_mspcg_match_dense_solution():
    L, Ls = (2, 2, 2, 4), 4
    A = O.Action(L, Ls, **MOB)
    U = synth.gauge_field(L, 0.5, 91)
    M = H.dense_of(lambda v: O.mdagm(A, U, v), (A.V // 2, Ls, 4, 3))
    rng = np.random.default_rng(13)
    b = H.rand_c(rng, (A.V // 2, Ls, 4, 3))
    exact = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, st = O.solve(A, U, b, tol=1e-11, maxiter=1000)
    assert st.converged and st.true_rel_resid <= 1e-11
    assert np.abs(x - exact).max() < 1e-8 * np.abs(exact).max()
    for k in (1, 3, 6):
        x, stp = O.solve(A, U, b, nblk=(1, 1, 1, 2), k=k, tol=1e-11, maxiter=1000)
        assert stp.converged and stp.true_rel_resid <= 1e-11
        assert np.abs(x - exact).max() < 1e-8 * np.abs(exact).max()
    # exact block solves (block-Jacobi PCG) need fewer outer iterations than CG
    _, stx = O.solve(A, U, b, nblk=(1, 1, 1, 2), k=300, tol=1e-11, maxiter=1000)
    assert stx.iters < st.iters


def test_solver_edge_cases():
    L, Ls = (2, 2, 2, 2), 4
    A = O.Action(L, Ls, **MOB)
    U = synth.gauge_field(L, 0.5, 92)
    b = np.zeros((A.V // 2, Ls, 4, 3), complex)
    x, st = O.solve(A, U, b)
    assert st.converged and st.iters == 0 and np.all(x == 0)
    rng = np.random.default_rng(14)
    b = H.rand_c(rng, b.shape)
    x, st = O.solve(A, U, b, maxiter=2)
    assert not st.converged and st.iters == 2
    # starting from the solution: no iteration needed
    xs, _ = O.solve(A, U, b, tol=1e-13)
    x, st = O.solve(A, U, b, x0=xs, tol=1e-10)
    assert st.iters == 0 and st.converged


def test_shamir_small_workload_converges():
    """The 4^4 x 8 Shamir workload: plain CG reaches 1e-10 true residual."""
    from paper_1811_08488_amd.workloads import WORKLOADS

    w = WORKLOADS["shamir_4x4x4x4_ls8"]
    A = O.Action(w.L, w.Ls, M5=w.M5, mf=w.mf, b=w.b, c=w.c)
    U = synth.gauge_field(w.L, w.eps, w.gauge_seed)
    phi = synth.source(w.L, w.Ls, 1, w.source_seed)[0]
    b, _ = O.prepare_rhs(A, U, phi)
    x, st = O.solve(A, U, b, tol=w.tol, maxiter=5000)
    assert st.converged and st.true_rel_resid <= w.tol
