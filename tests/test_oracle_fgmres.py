"""Pins of the oracle's FGMRES-DR (Sec. 4) against dense linear algebra and the invariants of
deflated restarting (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, solvers


def _normal_matrix(n, seed, small=()):
    """Normal matrix with eigenvalues 1..2 (+ small imaginary parts) and the given small
    eigenvalues, in a random unitary basis.  Returns (A, eigenvalues)."""
    rng = np.random.default_rng(seed)
    lam = 1.0 + rng.random(n) + 0.3j * (rng.random(n) - 0.5)
    lam[: len(small)] = small
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return Q @ np.diag(lam) @ Q.conj().T, lam


def _vector(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _krylov(A, r, m):
    """Orthonormal basis of span{r, A r, ..., A^m r} by QR of the power basis and the exact
    Hessenberg matrix V^H A V[:, :m] of that basis."""
    K = np.empty((r.size, m + 1), dtype=np.complex128)
    K[:, 0] = r / np.linalg.norm(r)
    for j in range(m):
        K[:, j + 1] = A @ K[:, j]
        K[:, j + 1] /= np.linalg.norm(K[:, j + 1])
    V, _ = np.linalg.qr(K)
    # fix the phases so that V[:, 0] is r / |r| exactly
    V[:, 0] *= np.vdot(V[:, 0], r) / abs(np.vdot(V[:, 0], r))
    return V, V.conj().T @ A @ V[:, :m]


def test_first_cycle_reaches_the_krylov_minimum():
    """Identity preconditioner: one cycle of length m gives min over x0 + K_m(A, r0) of |b - A x|."""
    n, m = 60, 6
    rng = np.random.default_rng(3)
    A = np.eye(n) + 0.4 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = _vector(n, 4)
    res = solvers.fgmres_dr(lambda v: A @ v, lambda v: v, b, tol=1e-300, m=m, k=0, maxit=m)
    K = np.empty((n, m), dtype=np.complex128)
    K[:, 0] = b
    for j in range(1, m):
        K[:, j] = A @ K[:, j - 1]
    Q, _ = np.linalg.qr(K)
    y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
    want = np.linalg.norm(b - A @ Q @ y) / np.linalg.norm(b)
    assert res.restarts == 1 and res.iters == m
    assert abs(res.history[1] - want) < 1e-10 * want


def test_harmonic_ritz_pairs_satisfy_their_definition():
    """y = V_m g, theta is a harmonic Ritz pair of A in span(V_m) iff A y - theta y is orthogonal
    to A V_m; checked with the dense A, not through the small-matrix formula."""
    n, m = 50, 8
    A, _ = _normal_matrix(n, 5, small=(0.01, 0.02 + 0.01j))
    A = A + 0.1 * np.triu(np.ones((n, n)), 1) / n  # not normal
    V, Hbar = _krylov(A, _vector(n, 6), m)
    theta, G = solvers.harmonic_ritz(Hbar)
    assert np.all(np.diff(np.abs(theta)) >= 0)
    AV = A @ V[:, :m]
    for i in range(m):
        y = V[:, :m] @ G[:, i]
        viol = np.linalg.norm(AV.conj().T @ (A @ y - theta[i] * y))
        assert viol < 1e-10 * np.linalg.norm(AV) * np.linalg.norm(A @ y)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_deflated_restart_keeps_the_arnoldi_relation(k):
    """After a deflated restart A Z = V Hbar still holds, V stays orthonormal and V c is the
    residual of the cycle (the theorem GMRES-DR rests on)."""
    n, m = 50, 8
    A, _ = _normal_matrix(n, 7, small=(0.01, 0.015j, 0.03))
    A = A + 0.1 * np.triu(np.ones((n, n)), 1) / n
    r = _vector(n, 8)
    V, Hbar = _krylov(A, r, m)
    # a flexible cycle: Z arbitrary (here a fixed nonsingular map of V), A Z = W Hbar for W
    # the basis of A Z: build it the same way as the Arnoldi of the flexible method
    M = np.eye(n) + 0.2 * np.diag(np.linspace(0, 1, n))
    Zm = M @ V[:, :m]
    W, _ = np.linalg.qr(np.column_stack([r, A @ Zm]))
    W[:, 0] *= np.vdot(W[:, 0], r) / abs(np.vdot(W[:, 0], r))
    Hf = W.conj().T @ A @ Zm
    assert np.linalg.norm(A @ Zm - W @ Hf) < 1e-12 * np.linalg.norm(A @ Zm)
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = np.linalg.norm(r)
    d = np.linalg.lstsq(Hf, c, rcond=None)[0]
    s = c - Hf @ d
    Vl = [W[:, i] for i in range(m + 1)]
    Zl = [Zm[:, i] for i in range(m)]
    Vn, Zn, Hn, cn, theta = solvers.deflate(Vl, Zl, Hf, s, k)
    Vn, Zn = np.column_stack(Vn), np.column_stack(Zn)
    assert Vn.shape == (n, k + 1) and Zn.shape == (n, k) and Hn.shape == (k + 1, k)
    assert np.linalg.norm(Vn.conj().T @ Vn - np.eye(k + 1)) < 1e-12
    assert np.linalg.norm(A @ Zn - Vn @ Hn) < 1e-10 * np.linalg.norm(A @ Zn)
    assert np.linalg.norm(Vn @ cn - W @ s) < 1e-12 * np.linalg.norm(W @ s)
    assert len(theta) == k


def test_linear_preconditioner_fgmres_equals_fgcr():
    """With a fixed linear preconditioner FGMRES (no deflation) and FGCR are the same method
    (Sec. 4): equal true residuals at every restart."""
    n, m = 80, 5
    A, _ = _normal_matrix(n, 9, small=(0.05,))
    A = A + 0.2 * np.triu(np.ones((n, n)), 1) / n
    rng = np.random.default_rng(10)
    Minv = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n))
    b = _vector(n, 11)
    op, pre = (lambda v: A @ v), (lambda v: Minv @ v)
    g = solvers.fgcr(op, pre, b, tol=1e-10, nkv=m)
    f = solvers.fgmres_dr(op, pre, b, tol=1e-10, m=m, k=0)
    assert g.converged and f.converged
    assert g.restarts == f.restarts and g.iters == f.iters
    for a, bb in zip(g.history, f.history):
        assert abs(a - bb) <= 1e-7 * a + 1e-13


def test_deflation_removes_small_eigenvalues():
    """Four tiny eigenvalues: restarted GMRES(10) crawls, GMRES-DR(10, 4) converges in far
    fewer matrix-vector products and its kept harmonic Ritz values are those eigenvalues."""
    n = 300
    small = np.array([1e-3, 2e-3 + 1e-3j, 3e-3, 4e-3 - 1e-3j])
    A, lam = _normal_matrix(n, 12, small=tuple(small))
    b = _vector(n, 13)
    op, pre = (lambda v: A @ v), (lambda v: v)
    plain = solvers.fgmres_dr(op, pre, b, tol=1e-10, m=10, k=0, maxit=3000)
    dr = solvers.fgmres_dr(op, pre, b, tol=1e-10, m=10, k=4, maxit=3000)
    assert dr.converged
    assert dr.iters < 0.4 * plain.iters
    assert np.linalg.norm(b - A @ dr.x) / np.linalg.norm(b) <= 1e-10
    got = np.sort_complex(dr.theta)
    want = np.sort_complex(small)
    assert np.abs(got - want).max() < 1e-6


def test_sap_fgmres_dr_4444_matches_dense_lu():
    """The smallest workload with the SAP preconditioner, restart 8 with 3 deflated vectors."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, 0.0, 1.0)
    b = synth.gaussian_spinor(dims)
    res = solvers.sap_fgmres_dr(U, A, b, (2, 2, 2, 2), nmr=4, ncy=5, m=8, k=3, tol=1e-10)
    assert res.converged
    assert dirac.norm(b - dirac.apply_D(U, A, res.x)) / dirac.norm(b) <= 1e-10
    M = dense.assemble(U, A)
    xd = sla.lu_solve(sla.lu_factor(M), b.ravel()).reshape(b.shape)
    assert dirac.norm(res.x - xd) / dirac.norm(xd) < np.linalg.cond(M) * 1e-10
