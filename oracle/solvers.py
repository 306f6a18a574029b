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
    describes ("on the internal border of the black blocks").

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


def fgcr(apply_op, precond, b, tol: float = 1e-10, nkv: int = 16, maxit: int = 10000, x0=None):
    """Restarted flexible GCR (Sec. 4), all in FP64.

    Each iteration k: phi_k = M(r); chi_k = D phi_k; orthogonalise chi_k against chi_0..chi_{k-1}
    by modified Gram-Schmidt (a_lk = <chi_l, chi_k>), normalise (b_k = |chi_k|), c_k = <chi_k, r>,
    r -= c_k chi_k.  The cycle ends after nkv iterations or when the recursive |r| <= tol |b| / 2;
    then the upper-triangular system b_k alpha_k + sum_{l>k} a_kl alpha_l = c_k gives the update
    x += sum alpha_k phi_k, and r = b - D x is recomputed.  The solve stops when the recomputed
    |r| / |b| <= tol, else the recursion restarts from that residual."""
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
        phis, chis = [], []
        a = np.zeros((nkv, nkv), dtype=np.complex128)
        bk = np.zeros(nkv)
        ck = np.zeros(nkv, dtype=np.complex128)
        k_done = 0
        for k in range(nkv):
            phi = precond(r)
            chi = apply_op(phi)
            for l in range(k):
                a[l, k] = dot(chis[l], chi)
                chi = chi - a[l, k] * chis[l]
            bk[k] = norm(chi)
            chi = chi / bk[k]
            ck[k] = dot(chi, r)
            r = r - ck[k] * chi
            phis.append(phi)
            chis.append(chi)
            k_done = k + 1
            iters += 1
            if norm(r) <= 0.5 * tol * bnorm or iters >= maxit:
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


def sap_fgcr(U, A, b, block, nmr=4, ncy=5, nkv=16, tol=1e-10, bc_t=1, maxit=10000, eo=False):
    """FGCR with the SAP preconditioner, the solver of Sec. 4, all FP64."""
    return fgcr(
        lambda v: apply_D(U, A, v, bc_t),
        lambda v: sap(U, A, v, block, nmr, ncy, bc_t, eo),
        b, tol=tol, nkv=nkv, maxit=maxit)
