"""Gauge-link derivatives of D_w and the pseudofermion force (oracle; test infrastructure only).

Sec. 1 of arXiv:1109.4279: the solves exist to give the HMC force that comes from the
fermion determinant.  For S = phi^dag (D^dag D)^-1 phi = |Y|^2 with Y = D^-dag phi and
X = D^-1 Y, a link variation U -> U + dU gives dS = -2 Re <Y, dD X>.

Two independent routes are kept here:

* ``link_grad`` - the analytic matrix K_mu(x) with d Re<Y, D X> = Re sum tr(dU_mu(x) K_mu(x))
  for an arbitrary complex variation dU: hopping terms from the operator directly, clover
  terms by the product rule over the four leaves of every plane that contain the link.
* ``force_bruteforce`` - the definition itself.  D is affine in any single link (a link
  appears at most once in each plaquette leaf and once in each hop), so
  dD X = D(U + T U e_link) X - D(U) X exactly; no finite step is involved.

The Lie-algebra force with generators T^a = i lambda_a / 2 is
    dS/d eps along U_mu(x) -> exp(eps T^a) U_mu(x)  =  -2 Re tr(T^a U K),
    F_mu(x) = sum_a (dS/d eps_a) T^a = TA(U_mu(x) K_mu(x)),
where TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6 (traceless anti-Hermitian part).
"""
from __future__ import annotations

import numpy as np

from .dirac import apply_D, clover_matrix, dag, mm, shift_links
from .gamma import GAMMA, ID4, sigma


def su3_generators() -> np.ndarray:
    """T^a = i lambda_a / 2 with the Gell-Mann matrices lambda_a, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return 0.5j * lam


def _shift_by(f: np.ndarray, offset) -> np.ndarray:
    """g(x) = f(x + offset) for a field with site axes 0..3."""
    for nu in range(4):
        if offset[nu]:
            f = shift_links(f, nu, offset[nu])
    return f


def _leaf_paths(rho: int, sig: int):
    """The four plaquettes of the clover leaf at y in the (rho, sigma) plane, as step lists
    (direction, +1 forward / -1 backward), all oriented rho -> sigma."""
    return [
        [(rho, 1), (sig, 1), (rho, -1), (sig, -1)],
        [(sig, 1), (rho, -1), (sig, -1), (rho, 1)],
        [(rho, -1), (sig, -1), (rho, 1), (sig, 1)],
        [(sig, -1), (rho, 1), (sig, 1), (rho, -1)],
    ]


def _walk(U: np.ndarray, path):
    """For a closed path starting at y return, per step, (matrix field W_i(y), link direction,
    offset of the link's site from y, dagger flag)."""
    pos = np.zeros(4, dtype=int)
    steps = []
    for d, s in path:
        if s > 0:
            site = pos.copy()
            pos[d] += 1
            w = _shift_by(U[d], site)
            steps.append((w, d, site, False))
        else:
            pos[d] -= 1
            site = pos.copy()
            w = dag(_shift_by(U[d], site))
            steps.append((w, d, site, True))
    assert not pos.any()
    return steps


def _outer(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sum over spin of a_t b_t^dag as a colour matrix: a, b shaped (..., 4, 3)."""
    return np.einsum("...ta,...tb->...ab", a, np.conj(b))


def link_grad(U: np.ndarray, X: np.ndarray, Y: np.ndarray, csw: float, bc_t: int = 1) -> np.ndarray:
    """K with d Re<Y, D X> = Re sum_{mu,x} tr(dU_mu(x) K_mu(x)); X, Y single spinor fields.

    The torch-convention gradient of Re<Y, D X> with respect to a complex U is K^dag."""
    K = np.zeros_like(U)
    L0 = U.shape[1]
    # hopping part: from site x (forward hop) and site x + mu (backward hop)
    for mu in range(4):
        Xp = _shift_by(X, [1 if n == mu else 0 for n in range(4)])
        Yp = _shift_by(Y, [1 if n == mu else 0 for n in range(4)])
        PmY = np.einsum("st,...tb->...sb", ID4 - GAMMA[mu], Y)
        PpYp = np.einsum("st,...tb->...sb", ID4 + GAMMA[mu], Yp)
        k = -0.5 * (_outer(Xp, PmY) + _outer(PpYp, X))
        if mu == 0 and bc_t != 1:
            k[L0 - 1] *= bc_t
        K[mu] += k
    if csw == 0:
        return K
    # clover part: Xi_{rs}(y) = (i c_sw / 16) (Gamma + Gamma^dag), Gamma_{rs} = sum sigma_st X_t Y_s^dag
    for rho in range(4):
        for sig in range(rho + 1, 4):
            gam = np.einsum("st,...ta,...sb->...ab", sigma(rho, sig), X, np.conj(Y))
            xi = (1j * csw / 16.0) * (gam + dag(gam))
            for path in _leaf_paths(rho, sig):
                steps = _walk(U, path)
                ws = [s[0] for s in steps]
                for i, (_, d, site, dg) in enumerate(steps):
                    r = mm(*(ws[i + 1:] + [xi] + ws[:i]))
                    if dg:
                        r = dag(r)
                    K[d] += _shift_by(r, -site)
    return K


def traceless_antihermitian(m: np.ndarray) -> np.ndarray:
    a = 0.5 * (m - dag(m))
    tr = np.trace(a, axis1=-2, axis2=-1)
    return a - (tr / 3.0)[..., None, None] * np.eye(3)


def lie_force(U: np.ndarray, K: np.ndarray) -> np.ndarray:
    """F_mu(x) = TA(U_mu(x) K_mu(x)) for K from ``link_grad`` of the pair (Y, X)."""
    return traceless_antihermitian(np.einsum("...ab,...bc->...ac", U, K))


def force_components(F: np.ndarray) -> np.ndarray:
    """Components dS/d eps_a of a force matrix: F = sum_a f_a T^a, tr(T^a T^b) = -delta/2."""
    T = su3_generators()
    return -2.0 * np.einsum("aij,...ji->...a", T, F).real


def force_bruteforce(U, m0, csw, X, Y, links, bc_t: int = 1) -> np.ndarray:
    """dS/d eps_a = -2 Re <Y, [D(U + T^a U e_link) - D(U)] X> for each (mu, site, a) in ``links``
    (site a 4-tuple), computed from the operator definition only."""
    T = su3_generators()
    A0 = clover_matrix(U, m0, csw)
    DX = apply_D(U, A0, X, bc_t)
    out = []
    for mu, site, a in links:
        Up = U.copy()
        idx = (mu,) + tuple(site)
        Up[idx] = U[idx] + T[a] @ U[idx]
        dDX = apply_D(Up, clover_matrix(Up, m0, csw), X, bc_t) - DX
        out.append(-2.0 * np.vdot(Y.ravel(), dDX.ravel()).real)
    return np.array(out)
