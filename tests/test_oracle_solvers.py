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


# Even/odd block solver: blocks of even volume (2x2x2x1) and of odd volume (3x3x1x1, where
# the even/odd split of a block depends on the parity of its corner).
EO_GEOMS = [((4, 4, 4, 2), (2, 2, 2, 1)), ((6, 6, 2, 2), (3, 3, 1, 1))]


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("colour", [0, 1])
@pytest.mark.parametrize("geom", EO_GEOMS)
def test_mr_eo_matches_dense_schur(geom, bc_t, colour):
    """Per block: partition the dense Dirichlet block matrix by site parity, form the Schur
    complement with library inverses, run textbook MR on it and rebuild the odd half."""
    dims, block = geom
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, -0.1, 1.0)
    eta = synth.gaussian_spinor(dims, seed=21)
    z, rho = solvers.mr_blocks_eo(U, A, eta, block, colour, 5, bc_t)
    MB = dense.assemble(U, A, bc_t, block=block)
    bid = dirac.block_index(dims, block).ravel()
    col = dirac.block_colour(dims, block).ravel()
    par = dirac.coords(dims).sum(-1).ravel() % 2
    zf, rf, ef = z.reshape(-1, 12), rho.reshape(-1, 12), eta.reshape(-1, 12)
    rows = lambda s: (s[:, None] * 12 + np.arange(12)).ravel()
    nblk = 0
    for b in np.unique(bid):
        sites = np.nonzero(bid == b)[0]
        if col[sites[0]] != colour:
            assert np.abs(zf[sites]).max() == 0 and np.abs(rf[sites]).max() == 0
            continue
        nblk += 1
        e, o = sites[par[sites] == 0], sites[par[sites] == 1]
        re_, ro = rows(e), rows(o)
        Mee, Meo = MB[np.ix_(re_, re_)], MB[np.ix_(re_, ro)]
        Moe, Moo = MB[np.ix_(ro, re_)], MB[np.ix_(ro, ro)]
        Moo_inv = np.linalg.inv(Moo)
        S = Mee - Meo @ Moo_inv @ Moe
        eta_e, eta_o = ef[e].ravel(), ef[o].ravel()
        ze, res = _textbook_mr(S, eta_e - Meo @ Moo_inv @ eta_o, 5)
        zo = Moo_inv @ (eta_o - Moe @ ze)
        scale = np.abs(ef).max()
        assert np.abs(zf[e].ravel() - ze).max() < 1e-13 * np.abs(ze).max()
        assert np.abs(zf[o].ravel() - zo).max() < 1e-13 * np.abs(zo).max()
        assert np.abs(rf[e].ravel() - res).max() < 1e-13 * scale
        assert np.abs(rf[o]).max() == 0
    assert nblk > 0


@pytest.mark.parametrize("bc_t", [1, -1])
def test_mr_eo_residual_is_block_residual(bc_t):
    """rho returned by the even/odd solver is eta - D_Lambda z on the solved blocks."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, -0.1, 1.0)
    eta = synth.gaussian_spinor(dims, seed=22)
    for colour in (0, 1):
        z, rho = solvers.mr_blocks_eo(U, A, eta, block, colour, 3, bc_t)
        on = (dirac.block_colour(dims, block) == colour)[..., None, None]
        want = np.where(on, eta - dirac.apply_D(U, A, z, bc_t, block), 0)
        assert np.abs(rho - want).max() < 1e-13 * np.abs(eta).max()
    # zero steps: z is the odd-site part of the exact solve with z_e = 0
    z0, rho0 = solvers.mr_blocks_eo(U, A, eta, block, 0, 0, bc_t)
    par = dirac.site_parity(dims)[..., None, None]
    assert np.abs(np.where(par == 0, z0, 0)).max() == 0


def test_mr_eo_beats_plain_mr(small):
    """At equal step count the Schur-complement iteration leaves a smaller block residual."""
    U, A = small
    eta = synth.gaussian_spinor(DIMS, seed=23)
    for nmr in (1, 2, 4):
        _, r_plain = solvers.mr_blocks(U, A, eta, BLOCK, 0, nmr)
        _, r_eo = solvers.mr_blocks_eo(U, A, eta, BLOCK, 0, nmr)
        assert dirac.norm(r_eo) < dirac.norm(r_plain)


@pytest.mark.parametrize("eo", [False, True])
@pytest.mark.parametrize("ncy", [1, 3])
def test_sap_exact_block_solves_closed_form(small, ncy, eo):
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
    got = solvers.sap(U, A, eta, BLOCK, nmr=60, ncy=ncy, eo=eo).ravel()
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()


def test_sap_is_a_good_preconditioner(small):
    U, A = small
    eta = synth.gaussian_spinor(DIMS, seed=14)
    psi = solvers.sap(U, A, eta, BLOCK, nmr=4, ncy=5)
    res = eta - dirac.apply_D(U, A, psi)
    assert dirac.norm(res) < 0.2 * dirac.norm(eta)


@pytest.mark.parametrize("eo", [False, True])
def test_fgcr_matches_dense_lu_4444(eo):
    """The smallest workload: 4^4, m0 = 0, c_sw = 1, 2^4 blocks, 4 MR steps x 5 SAP cycles,
    FGCR restart 8, tol 1e-10.  The answer must be the dense direct solve's within cond * tol."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, 0.0, 1.0)
    b = synth.gaussian_spinor(dims)
    res = solvers.sap_fgcr(U, A, b, (2, 2, 2, 2), nmr=4, ncy=5, nkv=8, tol=1e-10, eo=eo)
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


def test_fgcr_single_precision_basis_floor(small):
    """Iterative refinement (Sec. 4): a basis stored in single precision leaves the recursive
    residual and the true one parted by about the float rounding of the stored vectors, so
    one long cycle stops on a true residual near 1e-8 that an FP64 basis takes to 1e-14;
    the FP64 restarts still take the solve to the target."""
    U, A = small
    b = synth.gaussian_spinor(DIMS, seed=16)
    kw = dict(nmr=4, ncy=5, nkv=32, tol=1e-13)
    r64 = solvers.sap_fgcr(U, A, b, BLOCK, **kw)
    r32 = solvers.sap_fgcr(U, A, b, BLOCK, basis=np.complex64, **kw)
    assert r64.restarts == 1 and r64.history[1] <= 1e-13
    assert 1e-10 < r32.history[1] < 1e-6
    assert r32.converged and r32.restarts >= 2
    for res in (r64, r32):
        r = b - dirac.apply_D(U, A, res.x)
        assert dirac.norm(r) / dirac.norm(b) <= 1e-13


@pytest.mark.parametrize("basis", [np.complex128, np.complex64])
def test_fgcr_cycle_drop(small, basis):
    """drop = 1e-5: every restart before the last cuts the true residual by the drop (the
    recursive one by exactly that bound; an FP64 basis keeps the two equal to rounding, a
    single-precision one to its float floor, far below 1e-5 of the cycle's start), and the
    answer is the dense solve's within cond * tol."""
    U, A = small
    b = synth.gaussian_spinor(DIMS, seed=16)
    drop = 1e-5
    res = solvers.sap_fgcr(U, A, b, BLOCK, nmr=4, ncy=5, nkv=32, tol=1e-12, drop=drop, basis=basis)
    assert res.converged and res.restarts >= 3
    h = res.history
    slack = 1.0 + 1e-6 if basis is np.complex128 else 1.1
    for i in range(len(h) - 2):
        assert h[i + 1] <= drop * slack * h[i]
    r = b - dirac.apply_D(U, A, res.x)
    assert dirac.norm(r) / dirac.norm(b) <= 1e-12
    M = dense.assemble(U, A)
    xd = sla.lu_solve(sla.lu_factor(M), b.ravel()).reshape(b.shape)
    assert dirac.norm(res.x - xd) / dirac.norm(xd) < np.linalg.cond(M) * 1e-12
