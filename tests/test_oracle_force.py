"""Pins of the oracle's gauge-link derivative and pseudofermion force (no GPU).

* analytic product-rule derivative == the definition (D is affine in one link);
* force == central finite differences of S = |D^-dag phi|^2 computed by dense LU;
* gauge covariance of the force; the c_sw = 0 special case.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, force

TINY = (4, 2, 2, 2)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "force_fd_4x4x4x4.txt")


def _expm_su3(T):
    return sla.expm(T)


def test_D_is_affine_in_one_link():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims)
    X = synth.gaussian_spinor(dims, seed=21)
    dU = (np.random.default_rng(0).standard_normal((3, 3)) + 0j)
    idx = (1, 2, 3, 0, 1)
    out = []
    for t in (0.0, 1.0, 2.0):
        Ut = U.copy()
        Ut[idx] = U[idx] + t * dU
        out.append(dirac.apply_D(Ut, dirac.clover_matrix(Ut, -0.1, 1.0), X))
    assert np.abs(out[2] - 2 * out[1] + out[0]).max() < 1e-13


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("bc_t", [1, -1])
def test_link_grad_matches_definition(csw, bc_t):
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims)
    X = synth.gaussian_spinor(dims, seed=22)
    Y = synth.gaussian_spinor(dims, seed=23)
    K = force.link_grad(U, X, Y, csw, bc_t)
    comp = force.force_components(force.lie_force(U, K))
    rng = np.random.default_rng(5)
    links = []
    for _ in range(12):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(d)) for d in dims)
        links.append((mu, site, int(rng.integers(8))))
    # include links that cross the antiperiodic time face
    links += [(0, (3, 1, 0, 1), 2), (0, (3, 0, 1, 0), 7)]
    bf = force.force_bruteforce(U, -0.1, csw, X, Y, links, bc_t)
    an = np.array([comp[(mu,) + site + (a,)] for mu, site, a in links])
    assert np.abs(bf - an).max() < 1e-12 * np.abs(bf).max()


def test_link_grad_general_direction():
    """d Re<Y, D X> along an arbitrary complex dU equals Re tr(dU K)."""
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims)
    X = synth.gaussian_spinor(dims, seed=24)
    Y = synth.gaussian_spinor(dims, seed=25)
    K = force.link_grad(U, X, Y, 1.0, -1)
    rng = np.random.default_rng(6)
    A0 = dirac.clover_matrix(U, 0.3, 1.0)
    base = np.vdot(Y.ravel(), dirac.apply_D(U, A0, X, -1).ravel()).real
    for _ in range(6):
        idx = (int(rng.integers(4)),) + tuple(int(rng.integers(d)) for d in dims)
        dU = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Up = U.copy()
        Up[idx] = U[idx] + dU
        val = np.vdot(Y.ravel(), dirac.apply_D(Up, dirac.clover_matrix(Up, 0.3, 1.0), X, -1).ravel()).real
        want = np.trace(dU @ K[idx]).real
        assert abs((val - base) - want) < 1e-12 * max(1.0, abs(want))


def _oracle_force(U, m0, csw, phi, bc_t):
    A = dirac.clover_matrix(U, m0, csw)
    M = dense.assemble(U, A, bc_t)
    lu = sla.lu_factor(M)
    Y = sla.lu_solve(lu, phi.ravel(), trans=2).reshape(phi.shape)
    X = sla.lu_solve(lu, Y.ravel()).reshape(phi.shape)
    return force.lie_force(U, force.link_grad(U, X, Y, csw, bc_t))


@pytest.mark.parametrize("csw,bc_t", [(0.0, 1), (1.0, 1), (1.0, -1)])
def test_force_matches_finite_differences(csw, bc_t):
    dims = TINY
    m0 = -0.1
    U = synth.gauge_field(dims)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    F = force.force_components(_oracle_force(U, m0, csw, phi, bc_t))
    T = force.su3_generators()
    rng = np.random.default_rng(7)
    h = 1e-6
    fd, an = [], []
    for _ in range(10):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(d)) for d in dims)
        a = int(rng.integers(8))
        idx = (mu,) + site
        s = []
        for sign in (1, -1):
            Up = U.copy()
            Up[idx] = _expm_su3(sign * h * T[a]) @ U[idx]
            s.append(dense.action(Up, m0, csw, phi, bc_t))
        fd.append((s[0] - s[1]) / (2 * h))
        an.append(F[idx + (a,)])
    fd, an = np.array(fd), np.array(an)
    assert np.linalg.norm(fd - an) / np.linalg.norm(an) < 1e-6


def test_force_gauge_covariance():
    dims = TINY
    U = synth.gauge_field(dims)
    Om = synth.gauge_transform(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = dirac.mm(Om, U[mu], dirac.dag(dirac.shift_links(Om, mu, 1)))
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    phig = np.einsum("...ab,...sb->...sa", Om, phi)
    F = _oracle_force(U, -0.1, 1.0, phi, 1)
    Fg = _oracle_force(Ug, -0.1, 1.0, phig, 1)
    want = np.einsum("...ab,...bc,...dc->...ad", Om[None], F, np.conj(Om[None]))
    assert np.abs(Fg - want).max() < 1e-11 * np.abs(F).max()


def test_force_golden_finite_differences_4444():
    """Central differences of S on the 4^4 lattice (step 1e-6, 64 sampled link/generator
    triples), written by tests/golden/make_force_fd.py from the oracle's dense action."""
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file not generated")
    rows = np.loadtxt(GOLDEN)
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    F = force.force_components(_oracle_force(U, -0.1, 1.0, phi, 1))
    an = np.array([F[(int(r[0]), int(r[1]), int(r[2]), int(r[3]), int(r[4]), int(r[5]))] for r in rows])
    fd = rows[:, 6]
    assert np.linalg.norm(fd - an) / np.linalg.norm(an) < 1e-6
