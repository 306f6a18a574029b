"""GPU link derivative and pseudofermion force against the oracle and finite differences."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, force
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "force_fd_4x4x4x4.txt")


@pytest.mark.parametrize("csw,bc_t", [(0.0, 1), (1.0, 1), (1.0, -1)])
def test_link_grad_matches_oracle(csw, bc_t):
    dims, block = (8, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block, -0.1, csw, bc_t)
    X = synth.gaussian_spinor(dims, seed=51)
    Y = synth.gaussian_spinor(dims, seed=52)
    G = to_np(lat.link_grad(to_dev(Y), to_dev(X)))
    K = force.link_grad(gauge(dims), X, Y, csw, bc_t)
    Kd = np.conj(np.swapaxes(K, -1, -2))
    assert rel(G, Kd) < 1e-12


def test_link_grad_full_size_16c32():
    dims, block = (32, 16, 16, 16), (4, 4, 4, 4)
    lat = lattice(dims, block, -0.1, 1.0)
    X = synth.gaussian_spinor(dims, seed=53)
    Y = synth.gaussian_spinor(dims, seed=54)
    G = to_np(lat.link_grad(to_dev(Y), to_dev(X), coef=-2.0))
    K = force.link_grad(gauge(dims), X, Y, 1.0)
    assert rel(G, -2.0 * np.conj(np.swapaxes(K, -1, -2))) < 1e-12


@pytest.mark.parametrize("basis", ["f64", "f32"])
def test_force_4444_against_oracle_and_finite_differences(basis):
    """The force from the library's two solves (also with the single-precision recursion of
    an F32 basis: its FP64 restarts still reach 1e-13) against the dense-LU oracle force and
    the finite-difference golden file."""
    dims, block, m0, csw = (4, 4, 4, 4), (2, 2, 2, 2), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    F, Y, X, st = lat.force(to_dev(phi), tol=1e-13, sap_prec="f64", basis_prec=basis)
    F = to_np(F)
    U, A = gauge(dims), clover(dims, m0, csw)
    M = dense.assemble(U, A)
    lu = sla.lu_factor(M)
    Yd = sla.lu_solve(lu, phi.ravel(), trans=2).reshape(phi.shape)
    Xd = sla.lu_solve(lu, Yd.ravel()).reshape(phi.shape)
    Fo = force.lie_force(U, force.link_grad(U, Xd, Yd, csw))
    assert rel(F, Fo) < 1e-9
    # traceless anti-Hermitian
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() < 1e-14 * np.abs(F).max() + 1e-300
    if os.path.exists(GOLDEN):
        rows = np.loadtxt(GOLDEN)
        comp = force.force_components(F)
        an = np.array([comp[tuple(int(v) for v in r[:6])] for r in rows])
        assert np.linalg.norm(an - rows[:, 6]) / np.linalg.norm(rows[:, 6]) < 1e-6


@pytest.mark.parametrize("basis", ["f64", "f32"])
def test_force_16c32_solves_and_contraction(basis):
    """Force workload (16^3 x 32): both solves inside the force reach 1e-10, checked with the
    oracle's D, with either Krylov basis; the contraction itself is pinned by
    test_link_grad_full_size_16c32."""
    dims, block, m0, csw = (32, 16, 16, 16), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    F, Y, X, st = lat.force(to_dev(phi), tol=1e-10, sap_prec="f32", basis_prec=basis)
    U, A = gauge(dims), clover(dims, m0, csw)
    Y, X, F = to_np(Y), to_np(X), to_np(F)
    r1 = dirac.norm(phi - dirac.apply_Ddag(U, A, Y)) / dirac.norm(phi)
    r2 = dirac.norm(Y - dirac.apply_D(U, A, X)) / dirac.norm(Y)
    assert r1 <= 1e-10 and r2 <= 1e-10
    assert all(s["status"] == 0 for s in st)
