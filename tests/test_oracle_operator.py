"""Pins of the FP64 oracle's operator against mathematics it must satisfy (no GPU).

Each test fixes a part of the oracle by something other than the oracle itself:
Clifford algebra, gamma5-hermiticity, the free-field plane-wave closed form, gauge
covariance, the unit-gauge clover, and dense sub-matrices.
"""
import numpy as np
import pytest

import synth
from oracle import dense, dirac, gamma

SMALL = (4, 2, 2, 2)


def test_gamma_algebra():
    g = gamma.GAMMA
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * (m == n) * np.eye(4), atol=0)
    assert np.array_equal(gamma.GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))
    for m in range(4):
        for n in range(4):
            s = gamma.sigma(m, n)
            assert np.allclose(s, s.conj().T)
            assert np.allclose(s, -gamma.sigma(n, m))


def test_gauge_recipe_is_su3():
    U = synth.gauge_field((4, 4, 4, 4))
    eye = np.eye(3)
    assert np.abs(np.einsum("...ab,...cb->...ac", U, U.conj()) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # plaquette of the eps = 0.3, lambda/2 recipe (distinguishes it from the lambda normalisation)
    P = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            p = dirac.mm(U[mu], dirac.shift_links(U[nu], mu, 1), dirac.dag(dirac.shift_links(U[mu], nu, 1)),
                         dirac.dag(U[nu]))
            P += np.trace(p, axis1=-2, axis2=-1).real.mean() / 3.0
    assert 0.76 < P / 6 < 0.81


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("block", [None, (2, 2, 2, 2)])
def test_gamma5_hermiticity(bc_t, block):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, -0.1, 1.0)
    x = synth.gaussian_spinor(dims, seed=1)
    y = synth.gaussian_spinor(dims, seed=2)
    lhs = dirac.dot(y, dirac.apply_D(U, A, x, bc_t, block))
    rhs = dirac.dot(dirac.apply_Ddag(U, A, y, bc_t, block), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # and D is not Hermitian itself (the check above is not vacuous)
    assert abs(lhs - dirac.dot(dirac.apply_D(U, A, y, bc_t, block), x)) / abs(lhs) > 1e-3


def _free_symbol(p, m0):
    """D(p) = m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu for U = 1."""
    g = gamma.GAMMA
    return (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))


@pytest.mark.parametrize("bc_t", [1, -1])
def test_free_field_plane_waves(bc_t):
    dims = (4, 4, 2, 6)
    m0, csw = -0.3, 1.7
    U = synth.unit_gauge(dims)
    A = dirac.clover_matrix(U, m0, csw)
    x = dirac.coords(dims)
    rng = np.random.default_rng(3)
    for _ in range(6):
        n = [rng.integers(0, d) for d in dims]
        p = np.array([2 * np.pi * n[m] / dims[m] for m in range(4)], dtype=float)
        if bc_t == -1:
            p[0] = (2 * n[0] + 1) * np.pi / dims[0]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (x @ p))
        psi = phase[..., None, None] * u
        got = dirac.apply_D(U, A, psi, bc_t)
        want = phase[..., None, None] * (_free_symbol(p, m0) @ u)
        assert np.abs(got - want).max() < 1e-13


def _sorted(z):
    """Sort complex values by (real, imag) after rounding away last-bit noise."""
    return z[np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))]


@pytest.mark.parametrize("bc_t", [1, -1])
def test_free_field_spectrum_dense(bc_t):
    dims = SMALL
    m0 = 0.2
    U = synth.unit_gauge(dims)
    M = dense.assemble(U, dirac.clover_matrix(U, m0, 1.0), bc_t)
    ev = _sorted(np.linalg.eigvals(M))
    want = []
    for n in np.ndindex(*dims):
        p = np.array([2 * np.pi * n[m] / dims[m] for m in range(4)])
        if bc_t == -1:
            p[0] = (2 * n[0] + 1) * np.pi / dims[0]
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    want = _sorted(np.array(want))
    assert np.abs(ev - want).max() < 1e-12


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims)
    Om = synth.gauge_transform(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = dirac.mm(Om, U[mu], dirac.dag(dirac.shift_links(Om, mu, 1)))
    psi = synth.gaussian_spinor(dims, seed=5)
    opsi = np.einsum("...ab,...sb->...sa", Om, psi)
    for bc_t in (1, -1):
        A = dirac.clover_matrix(U, -0.1, 1.0)
        Ag = dirac.clover_matrix(Ug, -0.1, 1.0)
        lhs = dirac.apply_D(Ug, Ag, opsi, bc_t)
        rhs = np.einsum("...ab,...sb->...sa", Om, dirac.apply_D(U, A, psi, bc_t))
        assert np.abs(lhs - rhs).max() / np.abs(rhs).max() < 1e-13


def test_clover_properties():
    dims = (4, 4, 4, 4)
    m0, csw = -0.1, 1.0
    A1 = dirac.clover_matrix(synth.unit_gauge(dims), m0, csw)
    assert np.array_equal(A1, np.broadcast_to((4 + m0) * np.eye(12), A1.shape).astype(complex))
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, m0, csw)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-15
    # chiral structure: sigma_{mu nu} commutes with gamma5, so the clover has no
    # off-chirality blocks; its traceless part is odd in c_sw
    assert np.abs(A[..., :6, 6:]).max() == 0
    assert np.abs(A[..., 6:, :6]).max() == 0
    Am = dirac.clover_matrix(U, m0, -csw)
    assert np.abs((A + Am) / 2 - (4 + m0) * np.eye(12)).max() < 1e-15
    assert np.abs(A - (4 + m0) * np.eye(12)).max() > 1e-2


def test_field_strength_antisymmetry():
    U = synth.gauge_field((4, 4, 4, 4))
    F = dirac.field_strength(U)
    for mu in range(4):
        for nu in range(4):
            assert np.allclose(F[mu, nu], -F[nu, mu])
            assert np.abs(F[mu, nu] + dirac.dag(F[mu, nu])).max() < 1e-15


def test_clover_leaves_geometry():
    """Each leaf of Q_{mu nu} is a closed plaquette: on a pure-gauge field every leaf is 1."""
    dims = (4, 4, 4, 4)
    Om = synth.gauge_transform(dims)
    Ug = np.empty((4,) + dims + (3, 3), dtype=complex)
    for mu in range(4):
        Ug[mu] = dirac.mm(Om, dirac.dag(dirac.shift_links(Om, mu, 1)))
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                q = dirac.clover_leaves(Ug, mu, nu)
                assert np.abs(q - 4 * np.eye(3)).max() < 1e-13


def test_block_operator_is_dense_submatrix():
    dims = (4, 4, 2, 2)
    block = (2, 2, 1, 1)
    U = synth.gauge_field(dims)
    A = dirac.clover_matrix(U, -0.1, 1.0)
    for bc_t in (1, -1):
        M = dense.assemble(U, A, bc_t)
        MB = dense.assemble(U, A, bc_t, block)
        bid = np.repeat(dirac.block_index(dims, block).ravel(), 12)
        same = bid[:, None] == bid[None, :]
        assert np.array_equal(MB, np.where(same, M, 0))


def test_block_colouring():
    dims = (8, 4, 4, 4)
    col = dirac.block_colour(dims, (4, 2, 2, 2))
    for mu in range(4):
        nb = np.roll(col, -1, axis=mu)
        bid = dirac.block_index(dims, (4, 2, 2, 2))
        cross = bid != np.roll(bid, -1, axis=mu)
        # neighbouring blocks always have opposite colours (including across the periodic wrap)
        assert np.all(col[cross] != nb[cross])
    with pytest.raises(ValueError):
        dirac.check_blocking((12, 12, 12, 24), (4, 4, 4, 4))
    dirac.check_blocking((24, 12, 12, 12), (4, 2, 2, 2))


def test_field_strength_constant_flux():
    """Constant abelian flux Phi in the (mu, nu) plane: every leaf equals exp(i Phi) on the
    first two colours, so F = diag(i sin Phi, -i sin Phi, 0) exactly; a reversed leaf or a
    wrong normalisation would change it."""
    dims = (4, 4, 4, 4)
    x = dirac.coords(dims)
    for mu, nu in [(0, 1), (1, 3), (2, 0)]:
        phi = 2 * np.pi / 4
        U = synth.unit_gauge(dims)
        ang = phi * x[..., mu]
        U[nu][..., 0, 0] = np.exp(1j * ang)
        U[nu][..., 1, 1] = np.exp(-1j * ang)
        F = dirac.field_strength(U)
        want = np.diag([1j * np.sin(phi), -1j * np.sin(phi), 0])
        assert np.abs(F[mu, nu] - want).max() < 1e-15
        for a in range(4):
            for b in range(4):
                if {a, b} != {mu, nu}:
                    assert np.abs(F[a, b]).max() < 1e-15


def _flux_field(dims, mu, nu, phi):
    """Unit links except U_nu(x) = diag(e^{i phi x_mu}, e^{-i phi x_mu}, 1): a constant abelian
    flux phi through every (mu, nu) plaquette (L_mu phi must be a multiple of 2 pi)."""
    x = dirac.coords(dims)
    U = synth.unit_gauge(dims)
    U[nu][..., 0, 0] = np.exp(1j * phi * x[..., mu])
    U[nu][..., 1, 1] = np.exp(-1j * phi * x[..., mu])
    return U


def clover_flux_closed_form(mu, nu, phi, m0, csw):
    """The clover term on a constant abelian flux in the (mu, nu) plane.  There F_{mu nu} =
    i sin(phi) diag(1, -1, 0) and the other planes vanish (test_field_strength_constant_flux),
    and sigma_{nu mu} F_{nu mu} = sigma_{mu nu} F_{mu nu}, so the sum over ordered pairs is
    twice one term: A = (4 + m0) 1 + c_sw (i/2) sigma_{mu nu} (x) F_{mu nu}
                      = (4 + m0) 1 - (c_sw / 2) sin(phi) sigma_{mu nu} (x) diag(1, -1, 0),
    with sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] built from the (Clifford-pinned) gammas."""
    from oracle.gamma import GAMMA
    sig = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
    return (4 + m0) * np.eye(12) - 0.5 * csw * np.sin(phi) * np.kron(sig, np.diag([1.0, -1.0, 0.0]))


def test_clover_constant_flux_closed_form():
    """A constant abelian flux pins the clover coefficient c_sw (i/4), its sign and the factor
    two of the ordered sum: A equals the closed form at every site, and (basis-free) its
    spectrum is (4 + m0) +- (c_sw / 2) sin(phi), four times each, and (4 + m0) four times."""
    dims, m0, csw = (8, 8, 4, 8), -0.1, 1.3
    for mu, nu in [(0, 1), (0, 3), (1, 3), (3, 2)]:
        phi = 2 * np.pi * 3 / 8
        U = _flux_field(dims, mu, nu, phi)
        A = dirac.clover_matrix(U, m0, csw)
        want = clover_flux_closed_form(mu, nu, phi, m0, csw)
        assert np.abs(A - want).max() < 1e-14, (mu, nu)
        s = 0.5 * csw * np.sin(phi)
        ev = np.sort(np.linalg.eigvalsh(A[0, 0, 0, 0]))
        assert np.abs(ev - np.repeat([4 + m0 - s, 4 + m0, 4 + m0 + s], 4)).max() < 1e-14
