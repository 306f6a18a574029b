"""Pins of the oracle's block MR, SAP and FGCR against dense linear algebra (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, solvers

DIMS = (4, 4, 2, 2)
BLOCK = (2, 2, 1, 1)


@pytest.fixture(scope="module")
def small():
    U = synth.gauge_field(DIMS)
    A = dirac.clover_matrix(U, -0.1, 1.0)
    return U, A


def _textbook_mr(M, eta, nmr):
    z = np.zeros_like(eta)
    r = eta.copy()
    for _ in range(nmr):
        q = M @ r
        qq = np.vdot(q, q).real
        a = np.vdot(q, r) / qq
        z = z + a * r
        r = r - a * q
    return z, r


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("colour", [0, 1])
def test_mr_matches_dense_blockwise(small, bc_t, colour):
    U, A = small
    eta = synth.gaussian_spinor(DIMS, seed=11)
    z, rho = solvers.mr_blocks(U, A, eta, BLOCK, colour, 5, bc_t)
    M = dense.assemble(U, A, bc_t)
    bid = dirac.block_index(DIMS, BLOCK).ravel()
    col = dirac.block_colour(DIMS, BLOCK).ravel()
    zf, rf, ef = z.reshape(-1, 12), rho.reshape(-1, 12), eta.reshape(-1, 12)
    for b in np.unique(bid):
        sites = np.nonzero(bid == b)[0]
        rows = (sites[:, None] * 12 + np.arange(12)).ravel()
        if col[sites[0]] != colour:
            assert np.abs(zf[sites]).max() == 0 and np.abs(rf[sites]).max() == 0
            continue
        zz, rr = _textbook_mr(M[np.ix_(rows, rows)], ef[sites].ravel(), 5)
        assert np.abs(zf[sites].ravel() - zz).max() < 1e-13 * np.abs(zz).max()
        assert np.abs(rf[sites].ravel() - rr).max() < 1e-13 * np.abs(ef).max()


def test_mr_properties(small):
    U, A = small
    eta = synth.gaussian_spinor(DIMS, seed=12)
    norms = []
    for n in range(6):
        _, rho = solvers.mr_blocks(U, A, eta, BLOCK, 0, n)
        norms.append(dirac.norm(rho))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(norms, norms[1:]))
    assert norms[-1] < 0.5 * norms[0]
    z1, _ = solvers.mr_blocks(U, A, eta, BLOCK, 0, 4)
    z2, _ = solvers.mr_blocks(U, A, (2.5 - 1j) * eta, BLOCK, 0, 4)
    assert np.abs(z2 - (2.5 - 1j) * z1).max() < 1e-13 * np.abs(z2).max()


@pytest.mark.parametrize("ncy", [1, 3])
def test_sap_exact_block_solves_closed_form(small, ncy):
    """With MR run to convergence the SAP error propagator is [(1 - K1 D)(1 - K0 D)]^ncy with
    K_c the sum over colour-c blocks of the exact inverse Dirichlet block operators."""
    U, A = small
    M = dense.assemble(U, A)
    MB = dense.assemble(U, A, block=BLOCK)
    col = np.repeat(dirac.block_colour(DIMS, BLOCK).ravel(), 12)
    n = M.shape[0]
    K = []
    for c in (0, 1):
        P = np.diag((col == c).astype(float))
        sub = P @ MB @ P + np.diag((col != c).astype(float))
        K.append(P @ np.linalg.inv(sub) @ P)
    E = (np.eye(n) - K[1] @ M) @ (np.eye(n) - K[0] @ M)
    eta = synth.gaussian_spinor(DIMS, seed=13)
    want = (np.eye(n) - np.linalg.matrix_power(E, ncy)) @ np.linalg.solve(M, eta.ravel())
    got = solvers.sap(U, A, eta, BLOCK, nmr=60, ncy=ncy).ravel()
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()


def test_sap_is_a_good_preconditioner(small):
    U, A = small
    eta = synth.gaussian_spinor(DIMS, seed=14)
    psi = solvers.sap(U, A, eta, BLOCK, nmr=4, ncy=5)
    res = eta - dirac.apply_D(U, A, psi)
    assert dirac.norm(res) < 0.2 * dirac.norm(eta)


def test_fgcr_matches_dense_lu_4444():
    """The smallest workload: 4^4, m0 = 0, c_sw = 1, 2^4 blocks, 4 MR steps x 5 SAP cycles,
    FGCR restart 8, tol 1e-10.  The answer must be the dense direct solve's within cond * tol."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, 0.0, 1.0)
    b = synth.gaussian_spinor(dims)
    res = solvers.sap_fgcr(U, A, b, (2, 2, 2, 2), nmr=4, ncy=5, nkv=8, tol=1e-10)
    assert res.converged
    r = b - dirac.apply_D(U, A, res.x)
    assert dirac.norm(r) / dirac.norm(b) <= 1e-10
    M = dense.assemble(U, A)
    xd = sla.lu_solve(sla.lu_factor(M), b.ravel()).reshape(b.shape)
    cond = np.linalg.cond(M)
    assert dirac.norm(res.x - xd) / dirac.norm(xd) < cond * 1e-10
    assert res.iters < 40


def test_fgcr_restarts_and_maxit(small):
    U, A = small
    b = synth.gaussian_spinor(DIMS, seed=15)
    # restart length 2 forces several restarts; the solve still converges
    res = solvers.sap_fgcr(U, A, b, BLOCK, nmr=2, ncy=1, nkv=2, tol=1e-10)
    assert res.converged and res.restarts > 2
    r = b - dirac.apply_D(U, A, res.x)
    assert dirac.norm(r) / dirac.norm(b) <= 1e-10
    capped = solvers.sap_fgcr(U, A, b, BLOCK, nmr=2, ncy=1, nkv=2, tol=1e-10, maxit=3)
    assert not capped.converged and capped.iters == 3
