"""Wilson-Dirac operator with clover term, FP64 reference (oracle; test infrastructure only).

Follows the operator named in the abstract and Sec. 4 of arXiv:1109.4279 (the Wilson-Dirac
operator with clover term), which the paper does not write out.
The form used, with the paper silent on every convention, is

    D psi(x) = A(x) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                              + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ],

    A(x) = (4 + m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x),

with F the clover-leaf field strength (Q - Q^dag)/8, Q the sum of the four
plaquettes at x in the (mu, nu) plane all oriented mu -> nu, no trace
subtraction.  Fermion boundary conditions: periodic, or antiperiodic in time
(bc_t = -1 multiplies every hop that crosses the t = L0-1 -> 0 face by -1).

The Dirichlet block operator of Sec. 4 (blocks solved "with Dirichlet boundary
conditions") is D restricted to a block: every hop whose neighbour lies in a
different block is dropped, and the clover term is the full-lattice one.

Arrays follow ``synth``: U[4][L0][L1][L2][L3][3][3], spinors [..][L0..L3][4][3].
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, ID4, sigma

# ----------------------------------------------------------------------------- geometry


def lattice_dims(psi: np.ndarray) -> tuple:
    return tuple(psi.shape[-6:-2])


def shift_links(f: np.ndarray, nu: int, step: int) -> np.ndarray:
    """g(x) = f(x + step * nu_hat) for a link-like field with site axes 0..3 (periodic)."""
    return np.roll(f, -step, axis=nu)


def shift_spinor(f: np.ndarray, mu: int, step: int, bc_t: int = 1) -> np.ndarray:
    """g(x) = f(x + step * mu_hat) for a spinor field (site axes -6..-3), with the fermion
    boundary phase bc_t on the values that wrapped across the time boundary."""
    axis = f.ndim - 6 + mu
    g = np.roll(f, -step, axis=axis)
    if mu == 0 and bc_t != 1:
        g = g.copy()
        L0 = f.shape[axis]
        idx = [slice(None)] * f.ndim
        idx[axis] = L0 - 1 if step > 0 else 0
        g[tuple(idx)] *= bc_t
    return g


def coords(dims) -> np.ndarray:
    """Integer site coordinates, shape (L0, L1, L2, L3, 4)."""
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return np.stack(grids, axis=-1)


def block_index(dims, block) -> np.ndarray:
    """Lexicographic index of the block that contains each site, shape (L0..L3)."""
    x = coords(dims)
    nb = [dims[m] // block[m] for m in range(4)]
    bc = x // np.asarray(block)
    return ((bc[..., 0] * nb[1] + bc[..., 1]) * nb[2] + bc[..., 2]) * nb[3] + bc[..., 3]


def block_colour(dims, block) -> np.ndarray:
    """Chessboard colour of the block containing each site (Sec. 4): sum_mu floor(x_mu/b_mu) mod 2."""
    x = coords(dims)
    return (x // np.asarray(block)).sum(axis=-1) % 2


def site_parity(dims) -> np.ndarray:
    """Parity of each site, (x0 + x1 + x2 + x3) mod 2: 0 = even, 1 = odd.  Every
    nearest-neighbour hop inside a block joins an even and an odd site, since no block
    wraps around the lattice (the block count per axis is even)."""
    return coords(dims).sum(axis=-1) % 2


def same_block_mask(dims, block, mu: int, step: int) -> np.ndarray:
    """True where the neighbour x + step*mu_hat (periodic) lies in the same block as x."""
    bid = block_index(dims, block)
    return bid == np.roll(bid, -step, axis=mu)


def check_blocking(dims, block) -> None:
    """Blocks must tile the lattice and the block count along every axis must be even,
    otherwise periodic wrap-around makes two blocks of one colour touch."""
    for m in range(4):
        if block[m] <= 0 or dims[m] % block[m] or (dims[m] // block[m]) % 2:
            raise ValueError(f"block {block} does not give an even chessboard on {dims}")


def block_sum(f: np.ndarray, block) -> np.ndarray:
    """Sum of f over the sites of each block, broadcast back to every site of that block.
    f has site axes as its last four axes."""
    L = f.shape[-4:]
    shp = f.shape[:-4]
    split = []
    for m in range(4):
        split += [L[m] // block[m], block[m]]
    g = f.reshape(shp + tuple(split))
    s = g.sum(axis=(-7, -5, -3, -1), keepdims=True)
    return np.broadcast_to(s, g.shape).reshape(f.shape)


# ----------------------------------------------------------------------------- gauge algebra


def dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def mm(*ms: np.ndarray) -> np.ndarray:
    out = ms[0]
    for m in ms[1:]:
        out = out @ m
    return out


def clover_leaves(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): the four plaquettes at x in the (mu, nu) plane, each oriented mu -> nu."""
    Um, Un = U[mu], U[nu]

    def s(f, *steps):
        for d, k in steps:
            f = shift_links(f, d, k)
        return f

    l1 = mm(Um, s(Un, (mu, 1)), dag(s(Um, (nu, 1))), dag(Un))
    l2 = mm(Un, dag(s(Um, (mu, -1), (nu, 1))), dag(s(Un, (mu, -1))), s(Um, (mu, -1)))
    l3 = mm(dag(s(Um, (mu, -1))), dag(s(Un, (mu, -1), (nu, -1))), s(Um, (mu, -1), (nu, -1)), s(Un, (nu, -1)))
    l4 = mm(dag(s(Un, (nu, -1))), s(Um, (nu, -1)), s(Un, (mu, 1), (nu, -1)), dag(Um))
    return l1 + l2 + l3 + l4


def field_strength(U: np.ndarray) -> np.ndarray:
    """F_{mu nu}(x) = (Q_{mu nu} - Q_{mu nu}^dag) / 8, shape (4, 4, L0..L3, 3, 3); F_{mu mu} = 0."""
    dims = U.shape[1:5]
    F = np.zeros((4, 4) + tuple(dims) + (3, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            q = clover_leaves(U, mu, nu)
            f = (q - dag(q)) / 8.0
            F[mu, nu] = f
            F[nu, mu] = -f
    return F


def clover_matrix(U: np.ndarray, m0: float, csw: float) -> np.ndarray:
    """A(x) = (4 + m0) 1 + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} (x) F_{mu nu}(x) as a 12x12 matrix per
    site (row/column index 3*spin + colour), shape (L0..L3, 12, 12)."""
    dims = tuple(U.shape[1:5])
    F = field_strength(U)
    A = np.zeros(dims + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            A += np.einsum("st,...ab->...satb", sigma(mu, nu), F[mu, nu])
    A *= csw * 0.25j
    A = A.reshape(dims + (12, 12))
    A += (4.0 + m0) * np.eye(12)
    return A


def clover_inverse(A: np.ndarray) -> np.ndarray:
    """A(x)^-1 per site (the even/odd block solver needs it on the odd sites)."""
    return np.linalg.inv(A)


def chiral_blocks(A: np.ndarray) -> tuple:
    """The two 6x6 diagonal blocks of A in the chiral basis: spins (0, 1) and (2, 3)."""
    return A[..., :6, :6], A[..., 6:, 6:]


# ----------------------------------------------------------------------------- the operator


def apply_clover(A: np.ndarray, psi: np.ndarray) -> np.ndarray:
    flat = psi.reshape(psi.shape[:-2] + (12, 1))
    return (A @ flat).reshape(psi.shape)


def hop_terms(U: np.ndarray, psi: np.ndarray, bc_t: int = 1, block=None):
    """Yield (mu, forward, backward) with
    forward(x)  = (1 - gamma_mu) U_mu(x) psi(x + mu),
    backward(x) = (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu),
    hops into a different block zeroed when ``block`` is given."""
    dims = lattice_dims(psi)
    for mu in range(4):
        # spinors are (..., spin, colour): colour matrices act from the right as psi @ U^T,
        # spin matrices from the left as P @ psi
        pf = shift_spinor(psi, mu, +1, bc_t)
        fwd = (ID4 - GAMMA[mu]) @ (pf @ np.swapaxes(U[mu], -1, -2))
        w = psi @ np.conj(U[mu])
        bwd = (ID4 + GAMMA[mu]) @ shift_spinor(w, mu, -1, bc_t)
        if block is not None:
            fwd = fwd * same_block_mask(dims, block, mu, +1)[..., None, None]
            bwd = bwd * same_block_mask(dims, block, mu, -1)[..., None, None]
        yield mu, fwd, bwd


def apply_hop(U: np.ndarray, psi: np.ndarray, bc_t: int = 1, block=None) -> np.ndarray:
    """The hopping part of D: -1/2 sum_mu [forward + backward] (D = A + apply_hop)."""
    out = np.zeros_like(psi)
    for _, fwd, bwd in hop_terms(U, psi, bc_t, block):
        out = out - 0.5 * (fwd + bwd)
    return out


def apply_D(U: np.ndarray, A: np.ndarray, psi: np.ndarray, bc_t: int = 1, block=None) -> np.ndarray:
    """D_w psi (block=None) or the block-diagonal sum of the Dirichlet block operators D_Lambda psi."""
    out = apply_clover(A, psi)
    for _, fwd, bwd in hop_terms(U, psi, bc_t, block):
        out = out - 0.5 * (fwd + bwd)
    return out


def gamma5(psi: np.ndarray) -> np.ndarray:
    g = psi.copy()
    g[..., 2:, :] *= -1
    return g


def apply_Ddag(U, A, psi, bc_t: int = 1, block=None) -> np.ndarray:
    """D^dag psi = gamma5 D gamma5 psi (gamma5-hermiticity of D_w)."""
    return gamma5(apply_D(U, A, gamma5(psi), bc_t, block))


def dot(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a_i) b_i over every site, spin and colour component."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a: np.ndarray) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))
