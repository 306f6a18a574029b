"""Seeded synthetic inputs shared by the oracle-based tests, the GPU tests and the benchmark.

This module only draws random numbers and shapes them into gauge fields and
spinor sources.  It contains none of the solver's arithmetic (no Dirac
operator, no clover term, no Krylov or Schwarz step), so that the oracle and the
HIP path can both consume its output without sharing any of the method.

Conventions (stated once, used everywhere):

* A lattice is ``dims = (L0, L1, L2, L3)`` with axis 0 the time direction, the
  slowest array axis; sites are lexicographic with x3 fastest.
* A gauge field is a complex128 array ``U[4][L0][L1][L2][L3][3][3]``; ``U[mu]``
  at site x is the link from x to x + mu_hat.
* A spinor field is complex128 ``psi[...][L0][L1][L2][L3][4][3]`` (spin, then
  colour), with optional leading right-hand-side axes.

Gauge recipe: each link is exp(i * eps * H) with H = sum_a h_a lambda_a / 2,
h_a iid standard normal drawn in the order (mu, site, a), lambda_a the
Gell-Mann matrices; the exponential is taken through the eigendecomposition of
H and the result is re-unitarised (row 0 normalised, row 1 Gram-Schmidt
orthogonalised and normalised, row 2 = conj(row0 x row1)), which makes it an
SU(3) matrix to rounding.
"""
from __future__ import annotations

import numpy as np

GAUGE_SEED = 1234
RHS_SEED = 5678
GAUGE_TRANSFORM_SEED = 99
FORCE_PHI_SEED = 4321


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), normalised tr(l_a l_b) = 2 delta_ab."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def su3_generators() -> np.ndarray:
    """Anti-Hermitian generators T^a = i lambda_a / 2, shape (8, 3, 3); tr(T^a T^b) = -delta_ab / 2."""
    return 0.5j * gell_mann()


def reunitarise(m: np.ndarray) -> np.ndarray:
    """Project (..., 3, 3) near-unitary matrices to SU(3) by row Gram-Schmidt + cross product."""
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _expi_hermitian(h: np.ndarray, eps: float) -> np.ndarray:
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, np.conj(v))


def gauge_field(dims, eps: float = 0.3, seed: int = GAUGE_SEED, chunk: int = 1 << 20) -> np.ndarray:
    """Random near-identity SU(3) field U[4][L0][L1][L2][L3][3][3] (recipe in the module docstring)."""
    dims = tuple(int(d) for d in dims)
    vol = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    lam = gell_mann()
    out = np.empty((4, vol, 3, 3), dtype=np.complex128)
    for mu in range(4):
        hcoef = rng.standard_normal((vol, 8))
        for s0 in range(0, vol, chunk):
            s1 = min(vol, s0 + chunk)
            h = np.einsum("sa,aij->sij", hcoef[s0:s1], lam) * 0.5
            out[mu, s0:s1] = reunitarise(_expi_hermitian(h, eps))
    return out.reshape((4,) + dims + (3, 3))


def unit_gauge(dims) -> np.ndarray:
    dims = tuple(int(d) for d in dims)
    u = np.zeros((4,) + dims + (3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gauge_transform(dims, seed: int = GAUGE_TRANSFORM_SEED) -> np.ndarray:
    """A random SU(3) matrix per site, Omega[L0][L1][L2][L3][3][3] (Haar-ish via QR + phase fix)."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(dims + (3, 3)) + 1j * rng.standard_normal(dims + (3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[..., None, None]
    return reunitarise(q)


def gaussian_spinor(dims, nrhs: int | None = None, seed: int = RHS_SEED) -> np.ndarray:
    """Gaussian complex source(s): Re and Im iid N(0,1), drawn as one array [nrhs][V][4][3][2]."""
    dims = tuple(int(d) for d in dims)
    vol = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    n = 1 if nrhs is None else int(nrhs)
    raw = rng.standard_normal((n, vol, 4, 3, 2))
    psi = (raw[..., 0] + 1j * raw[..., 1]).reshape((n,) + dims + (4, 3))
    return psi[0] if nrhs is None else psi


def point_sources(dims) -> np.ndarray:
    """The 12 spin-colour point sources at the origin, index 3*s + c, shape [12][L0..L3][4][3]."""
    dims = tuple(int(d) for d in dims)
    psi = np.zeros((12,) + dims + (4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            psi[(3 * s + c, 0, 0, 0, 0, s, c)] = 1.0
    return psi
