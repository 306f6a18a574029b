"""Block MR, Schwarz alternating procedure and restarted FGCR in FP64 (oracle; test
infrastructure only).

These are iterations, not closed forms, so they follow the steps of Sec. 4 of
arXiv:1109.4279 in order; the readings taken where the paper is silent are
stated per function.  Inner products are <a, b> = sum conj(a) b.
"""
from __future__ import annotations

import numpy as np

from .dirac import (apply_clover, apply_D, apply_hop, block_colour, block_sum, check_blocking, clover_inverse,
                    dot, lattice_dims, norm, site_parity)


def mr_blocks(U, A, eta, block, colour: int, nmr: int, bc_t: int = 1):
    """Minimal-residual block solver of Sec. 4: on every block of the given chessboard colour,
    nmr MR steps on the Dirichlet block operator from a zero start,

        q = D_Lambda rho,  alpha = <q, rho> / <q, q>,  z += alpha rho,  rho -= alpha q,

    with alpha computed per block.  A block whose <q, q> is zero keeps alpha = 0.
    Returns (z, rho), both zero outside the blocks of that colour."""
    dims = lattice_dims(eta)
    mask = (block_colour(dims, block) == colour)[..., None, None]
    rho = np.where(mask, eta, 0)
    z = np.zeros_like(rho)
    for _ in range(nmr):
        q = np.where(mask, apply_D(U, A, rho, bc_t, block), 0)
        qr = block_sum(np.sum(np.conj(q) * rho, axis=(-2, -1)), block)
        qq = block_sum(np.sum(np.abs(q) ** 2, axis=(-2, -1)), block)
        safe = np.where(qq > 0, qq, 1.0)
        alpha = np.where(qq > 0, qr / safe, 0.0)[..., None, None]
        z = z + alpha * rho
        rho = rho - alpha * q
    return z, rho


def mr_blocks_eo(U, A, eta, block, colour: int, nmr: int, bc_t: int = 1, Ainv=None):
    """Even/odd-preconditioned block solver (Sec. 4, Table 1: even/odd preconditioning is
    used inside the block solver).  On a block the sites split by parity into e and o and
    the Dirichlet block operator is [[A_ee, H_eo], [H_oe, A_oo]] with H its in-block hops.
    Eliminating the odd sites leaves, on the even sites, the Schur complement

        S = A_ee - H_eo A_oo^-1 H_oe,   S z_e = eta_e - H_eo A_oo^-1 eta_o.

    nmr MR steps (as in ``mr_blocks``, alpha per block) on S from z_e = 0 give z_e; the odd
    half follows exactly, z_o = A_oo^-1 (eta_o - H_oe z_e).  The MR residual of S is the
    block residual eta - D_Lambda z on the even sites, and that residual is zero on the odd
    ones.  Returns (z, rho), both zero outside the blocks of that colour."""
    dims = lattice_dims(eta)
    if Ainv is None:
        Ainv = clover_inverse(A)
    on = (block_colour(dims, block) == colour)[..., None, None]
    par = site_parity(dims)[..., None, None]
    ev = on & (par == 0)
    od = on & (par == 1)

    def hop(v, dst):  # in-block hops into the sites of mask dst
        return np.where(dst, apply_hop(U, v, bc_t, block), 0)

    def schur(v):  # v lives on the even sites
        w = apply_clover(Ainv, hop(v, od))
        return np.where(ev, apply_clover(A, v), 0) - hop(w, ev)

    eta_e = np.where(ev, eta, 0)
    t_o = np.where(od, apply_clover(Ainv, np.where(od, eta, 0)), 0)
    rho = eta_e - hop(t_o, ev)
    z = np.zeros_like(rho)
    for _ in range(nmr):
        q = schur(rho)
        qr = block_sum(np.sum(np.conj(q) * rho, axis=(-2, -1)), block)
        qq = block_sum(np.sum(np.abs(q) ** 2, axis=(-2, -1)), block)
        safe = np.where(qq > 0, qq, 1.0)
        alpha = np.where(qq > 0, qr / safe, 0.0)[..., None, None]
        z = z + alpha * rho
        rho = rho - alpha * q
    z_o = np.where(od, apply_clover(Ainv, np.where(od, eta, 0) - hop(z, od)), 0)
    return z + z_o, rho


def sap(U, A, eta, block, nmr: int, ncy: int, bc_t: int = 1, eo: bool = False):
    """Schwarz alternating procedure of Sec. 4 used as a preconditioner: psi = 0 and rho = eta
    at the start; each cycle solves the white (colour 0) blocks, then the black ones, on the
    current residual, adds the block solutions to psi and updates the residual.

    The residual update is written as its definition rho <- rho - D z: z lives on the blocks
    just solved, so this leaves the MR residual on those blocks and subtracts the hops out of
    them on the border sites of the opposite-colour blocks, which is the update the paper
    describes for the sites just inside the other colour's blocks.

    eo selects the even/odd-preconditioned block solver ``mr_blocks_eo``."""
    check_blocking(lattice_dims(eta), block)
    psi = np.zeros_like(eta)
    rho = eta.copy()
    Ainv = clover_inverse(A) if eo else None
    for _ in range(ncy):
        for colour in (0, 1):
            if eo:
                z, _ = mr_blocks_eo(U, A, rho, block, colour, nmr, bc_t, Ainv)
            else:
                z, _ = mr_blocks(U, A, rho, block, colour, nmr, bc_t)
            psi = psi + z
            rho = rho - apply_D(U, A, z, bc_t)
    return psi


class FGCRResult:
    def __init__(self, x, converged, iters, restarts, history):
        self.x = x
        self.converged = converged
        self.iters = iters
        self.restarts = restarts
        self.history = history


def fgcr(apply_op, precond, b, tol: float = 1e-10, nkv: int = 16, maxit: int = 10000, x0=None,
         drop: float = 0.0, basis=np.complex128):
    """Restarted flexible GCR (Sec. 4), in FP64 arithmetic.

    Each iteration k: phi_k = M(r); chi_k = D phi_k; orthogonalise chi_k against chi_0..chi_{k-1}
    by modified Gram-Schmidt (a_lk = <chi_l, chi_k>), normalise (b_k = |chi_k|), c_k = <chi_k, r>,
    r -= c_k chi_k.  The cycle ends after nkv iterations or when the recursive |r| <= tol |b| / 2;
    then the upper-triangular system b_k alpha_k + sum_{l>k} a_kl alpha_l = c_k gives the update
    x += sum alpha_k phi_k, and r = b - D x is recomputed.  The solve stops when the recomputed
    |r| / |b| <= tol, else the recursion restarts from that residual.

    Iterative refinement (Sec. 4: the recursion in single precision, the residual and the
    solution in double precision at each restart), in the reading taken here: D phi_k, the
    normalised chi_k and the recursive residual are held in `basis` (np.complex64 for single
    precision: each component rounded; the residual when the cycle takes over the recomputed
    one and after every update) and the residual is updated with chi_k as held, so that
    what the recursion stores carries the single precision and the Gram-Schmidt arithmetic
    stays double; with drop > 0 a cycle also ends once the recursive |r| <= drop times the
    recomputed |r| it started from."""
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_op(x) if x0 is not None else b.copy()
    history = [norm(r) / bnorm]
    iters = 0
    restarts = 0
    while True:
        if history[-1] <= tol:
            return FGCRResult(x, True, iters, restarts, history)
        if iters >= maxit:
            return FGCRResult(x, False, iters, restarts, history)
        r_start = norm(r)
        r = r.astype(basis).astype(np.complex128)
        phis, chis = [], []
        a = np.zeros((nkv, nkv), dtype=np.complex128)
        bk = np.zeros(nkv)
        ck = np.zeros(nkv, dtype=np.complex128)
        k_done = 0
        for k in range(nkv):
            phi = precond(r)
            chi = apply_op(phi).astype(basis).astype(np.complex128)
            for l in range(k):
                a[l, k] = dot(chis[l], chi)
                chi = chi - a[l, k] * chis[l]
            bk[k] = norm(chi)
            chi = chi / bk[k]
            ck[k] = dot(chi, r)
            chi = chi.astype(basis).astype(np.complex128)
            r = (r - ck[k] * chi).astype(basis).astype(np.complex128)
            phis.append(phi)
            chis.append(chi)
            k_done = k + 1
            iters += 1
            rn = norm(r)
            if rn <= 0.5 * tol * bnorm or rn <= drop * r_start or iters >= maxit:
                break
        alpha = np.zeros(k_done, dtype=np.complex128)
        for k in range(k_done - 1, -1, -1):
            s = ck[k] - sum(a[k, l] * alpha[l] for l in range(k + 1, k_done))
            alpha[k] = s / bk[k]
        for k in range(k_done):
            x = x + alpha[k] * phis[k]
        r = b - apply_op(x)
        restarts += 1
        history.append(norm(r) / bnorm)


def sap_fgcr(U, A, b, block, nmr=4, ncy=5, nkv=16, tol=1e-10, bc_t=1, maxit=10000, eo=False, drop=0.0,
             basis=np.complex128):
    """FGCR with the SAP preconditioner, the solver of Sec. 4, in FP64 arithmetic (with
    `basis` and `drop` as in fgcr)."""
    return fgcr(
        lambda v: apply_D(U, A, v, bc_t),
        lambda v: sap(U, A, v, block, nmr, ncy, bc_t, eo),
        b, tol=tol, nkv=nkv, maxit=maxit, drop=drop, basis=basis)


def harmonic_ritz(Hbar: np.ndarray):
    """Harmonic Ritz pairs of a cycle of m Arnoldi steps (Sec. 4) from the (m+1) x m upper
    Hessenberg matrix Hbar: with H its top m x m block and h = Hbar[m, m-1], the pairs are
    the eigenpairs of H + |h|^2 H^-H e_m e_m^T.  Returns (theta, G) with the columns of G
    the eigenvectors, sorted by increasing |theta|."""
    m = Hbar.shape[1]
    H = Hbar[:m, :m]
    em = np.zeros(m, dtype=np.complex128)
    em[-1] = 1.0
    f = np.linalg.solve(H.conj().T, em)
    Hh = H + abs(Hbar[m, m - 1]) ** 2 * np.outer(f, em)
    theta, G = np.linalg.eig(Hh)
    order = np.argsort(np.abs(theta), kind="stable")
    return theta[order], G[:, order]


def _orthonormalise(cols):
    """Modified Gram-Schmidt on a list of vectors; returns the matrix of orthonormal columns."""
    out = []
    for v in cols:
        w = v.astype(np.complex128).copy()
        for q in out:
            w = w - np.vdot(q, w) * q
        out.append(w / np.linalg.norm(w))
    return np.stack(out, axis=1)


def deflation_basis(Hbar: np.ndarray, s: np.ndarray, k: int):
    """The (m+1) x (k+1) matrix P of a deflated restart: the k harmonic Ritz vectors of
    smallest |theta| padded with a zero, then the least-squares residual s, orthonormalised
    in that order.  Returns (P, theta[:k])."""
    theta, G = harmonic_ritz(Hbar)
    cols = [np.append(G[:, i], 0.0) for i in range(k)] + [s]
    return _orthonormalise(cols), theta[:k]


def deflate(V, Z, Hbar, s, k: int):
    """Restart state from k harmonic Ritz vectors: V <- V P, Z <- Z P[:m, :k],
    Hbar <- P^H Hbar P[:m, :k], c <- P^H s.  Returns (V, Z, Hbar, c, theta)."""
    m = Hbar.shape[1]
    P, theta = deflation_basis(Hbar, s, k)
    Vn = [sum(P[i, l] * V[i] for i in range(m + 1)) for l in range(k + 1)]
    Zn = [sum(P[i, l] * Z[i] for i in range(m)) for l in range(k)]
    return Vn, Zn, P.conj().T @ Hbar @ P[:m, :k], P.conj().T @ s, theta


class FGMRESDRResult(FGCRResult):
    def __init__(self, x, converged, iters, restarts, history, theta):
        super().__init__(x, converged, iters, restarts, history)
        self.theta = theta  # harmonic Ritz values kept at the last deflated restart


def fgmres_dr(apply_op, precond, b, tol: float = 1e-10, m: int = 16, k: int = 0, maxit: int = 10000, x0=None):
    """Restarted flexible GMRES with deflated restarts, all in FP64 (Sec. 4: FGMRES-DR, the
    flexible form of Morgan's GMRES-DR).

    A cycle extends an orthonormal basis v_0.. with a variable preconditioner: z_j = M(v_j),
    w = A z_j, orthogonalised against every v_i by modified Gram-Schmidt (h_ij = <v_i, w>),
    h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}; so A Z = V Hbar.  The residual is V c, c its
    coefficients; the cycle ends after m vectors z or once min_d |c - Hbar d| <= tol |b| / 2.
    Then x += Z d for the least-squares d and r = b - A x is recomputed; the solve stops when
    |r| / |b| <= tol.

    Restart: with k = 0 the next cycle starts from v_0 = r / |r| (restarted FGMRES).  With
    k > 0 the k harmonic Ritz vectors of smallest |theta| (``harmonic_ritz``), padded with a
    zero, are orthonormalised, the least-squares residual s = c - Hbar d is orthonormalised
    against them, and these k+1 columns P give the next cycle's start: V <- V P,
    Z <- Z P[:m, :k], Hbar <- P^H Hbar P[:m, :k], c <- P^H s.  The cycle then extends the
    basis from k+1 to m+1 vectors."""
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_op(x) if x0 is not None else b.copy()
    history = [norm(r) / bnorm]
    iters = 0
    restarts = 0
    theta_kept = None
    V, Z, Hbar, c = [], [], None, None
    while True:
        if history[-1] <= tol:
            return FGMRESDRResult(x, True, iters, restarts, history, theta_kept)
        if iters >= maxit:
            return FGMRESDRResult(x, False, iters, restarts, history, theta_kept)
        if not V:  # plain start from the residual
            beta = norm(r)
            V = [r / beta]
            Z = []
            Hbar = np.zeros((1, 0), dtype=np.complex128)
            c = np.zeros(1, dtype=np.complex128)
            c[0] = beta
        d = np.zeros(0, dtype=np.complex128)
        while len(Z) < m and iters < maxit:
            j = len(Z)
            z = precond(V[j])
            w = apply_op(z)
            h = np.zeros(j + 2, dtype=np.complex128)
            for i in range(j + 1):
                h[i] = dot(V[i], w)
                w = w - h[i] * V[i]
            h[j + 1] = norm(w)
            Z.append(z)
            V.append(w / h[j + 1])
            Hn = np.zeros((j + 2, j + 1), dtype=np.complex128)
            Hn[: j + 1, :j] = Hbar
            Hn[:, j] = h
            Hbar = Hn
            c = np.append(c, 0.0)
            iters += 1
            d = np.linalg.lstsq(Hbar, c, rcond=None)[0]
            if np.linalg.norm(c - Hbar @ d) <= 0.5 * tol * bnorm:
                break
        for j in range(len(Z)):
            x = x + d[j] * Z[j]
        r = b - apply_op(x)
        restarts += 1
        history.append(norm(r) / bnorm)
        s = c - Hbar @ d
        mm = len(Z)
        kk = min(k, mm - 1)
        if kk <= 0:
            V = []
            continue
        V, Z, Hbar, c, theta_kept = deflate(V, Z, Hbar, s, kk)


def sap_fgmres_dr(U, A, b, block, nmr=4, ncy=5, m=16, k=0, tol=1e-10, bc_t=1, maxit=10000, eo=False):
    """FGMRES-DR with the SAP preconditioner (Sec. 4), all FP64."""
    return fgmres_dr(
        lambda v: apply_D(U, A, v, bc_t),
        lambda v: sap(U, A, v, block, nmr, ncy, bc_t, eo),
        b, tol=tol, m=m, k=k, maxit=maxit)
