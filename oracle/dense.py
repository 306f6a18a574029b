"""Dense-matrix brute force on tiny lattices (oracle; test infrastructure only).

The operator D_w is assembled column by column from ``dirac.apply_D`` so that direct
solves (LU), spectra and block sub-matrices can be taken with library routines.  The
row/column index is lexicographic (site, spin, colour) with colour fastest.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dirac import apply_D, clover_matrix


def assemble(U, A, bc_t: int = 1, block=None, chunk: int = 768) -> np.ndarray:
    dims = tuple(U.shape[1:5])
    n = int(np.prod(dims)) * 12
    M = np.empty((n, n), dtype=np.complex128)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        e = np.zeros((c1 - c0, n), dtype=np.complex128)
        e[np.arange(c1 - c0), np.arange(c0, c1)] = 1.0
        cols = apply_D(U, A, e.reshape((c1 - c0,) + dims + (4, 3)), bc_t, block)
        M[:, c0:c1] = cols.reshape(c1 - c0, n).T
    return M


def solve(U, A, b, bc_t: int = 1) -> np.ndarray:
    """x = D^-1 b by dense LU."""
    M = assemble(U, A, bc_t)
    x = sla.lu_solve(sla.lu_factor(M), b.reshape(-1))
    return x.reshape(b.shape)


def action(U, m0: float, csw: float, phi, bc_t: int = 1) -> float:
    """S = phi^dag (D^dag D)^-1 phi = |D^-dag phi|^2 by dense LU."""
    M = assemble(U, clover_matrix(U, m0, csw), bc_t)
    y = sla.lu_solve(sla.lu_factor(M), phi.reshape(-1), trans=2)
    return float(np.vdot(y, y).real)
