"""torch.autograd around D, the solve and the pseudofermion action: gradcheck in FP64 and the
adjoint identity; the U-gradient of the action matches the oracle force."""
import numpy as np
import pytest

import synth
from oracle import dense, dirac, force
from tests.helpers import gauge, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

DIMS, BLOCK = (2, 2, 2, 2), (1, 1, 1, 1)


def _inputs(seed=61):
    import torch
    U = to_dev(gauge(DIMS)).requires_grad_(True)
    x = to_dev(synth.gaussian_spinor(DIMS, seed=seed)).requires_grad_(True)
    return torch, U, x


def test_dirac_apply_gradcheck():
    from paper_1109_4279_amd.autograd import dirac_apply
    torch, U, x = _inputs()
    f = lambda U_, x_: dirac_apply(U_, x_, block=BLOCK, m0=-0.1, csw=1.0, bc_t=-1)
    assert torch.autograd.gradcheck(f, (U, x), eps=1e-6, atol=1e-7, rtol=1e-6, fast_mode=True)


@pytest.mark.parametrize("eo", [0, 1])
def test_dirac_solve_gradcheck(eo):
    """Through the solve with either block solver (single-site blocks: with even/odd the
    block solve is the exact inverse of the site's clover term on both parities)."""
    from paper_1109_4279_amd.autograd import dirac_solve
    torch, U, b = _inputs(62)
    f = lambda U_, b_: dirac_solve(U_, b_, block=BLOCK, m0=0.2, csw=1.0, tol=1e-14, maxit=400,
                                   sap_prec="f64", nkv=12, eo=eo)
    assert torch.autograd.gradcheck(f, (U, b), eps=1e-5, atol=1e-6, rtol=1e-5, fast_mode=True)


def test_adjoint_identity_4444():
    """<dy, D x> = <D^dag dy, x> through the autograd backward."""
    import torch
    from paper_1109_4279_amd.autograd import dirac_apply
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = to_dev(gauge(dims))
    x = to_dev(synth.gaussian_spinor(dims, seed=63)).requires_grad_(True)
    dy = to_dev(synth.gaussian_spinor(dims, seed=64))
    y = dirac_apply(U, x, block=block, m0=-0.1, csw=1.0)
    (gx,) = torch.autograd.grad(y, x, dy)
    lhs = torch.vdot(dy.flatten(), y.flatten())
    rhs = torch.vdot(gx.flatten(), x.flatten())
    assert abs((lhs - rhs).item()) < 1e-12 * abs(lhs.item())


def test_action_gradient_matches_oracle_force():
    import torch
    from paper_1109_4279_amd.autograd import pseudofermion_action
    dims, block, m0, csw = (4, 4, 4, 4), (2, 2, 2, 2), -0.1, 1.0
    Un = gauge(dims)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    U = to_dev(Un).requires_grad_(True)
    S = pseudofermion_action(U, to_dev(phi), block=block, m0=m0, csw=csw, tol=1e-13, sap_prec="f64")
    (G,) = torch.autograd.grad(S, U)
    G = to_np(G)
    # oracle: S by dense LU, force from its solutions
    A = dirac.clover_matrix(Un, m0, csw)
    M = dense.assemble(Un, A)
    import scipy.linalg as sla
    lu = sla.lu_factor(M)
    Y = sla.lu_solve(lu, phi.ravel(), trans=2).reshape(phi.shape)
    X = sla.lu_solve(lu, Y.ravel()).reshape(phi.shape)
    assert abs(S.item() - np.vdot(Y, Y).real) < 1e-9 * abs(S.item())
    K = force.link_grad(Un, X, Y, csw)
    assert rel(G, -2.0 * np.conj(np.swapaxes(K, -1, -2))) < 1e-9
    # the Lie-algebra projection of the torch gradient is the force: dS = Re tr(dU G^dag),
    # so d S / d eps_a = Re tr(T^a U G^dag) and F = sum_a (dS/d eps_a) T^a = -TA(U G^dag) / 2
    F = -0.5 * force.traceless_antihermitian(np.einsum("...ab,...cb->...ac", Un, np.conj(G)))
    Fo = force.lie_force(Un, K)
    assert rel(F, Fo) < 1e-9


@pytest.mark.timeout(300)
def test_action_gradient_16c32_matches_the_force():
    """16^3 x 32 (the force workload): the autograd gradient of the pseudofermion action,
    projected on the Lie algebra, equals the library's force, and the action the library
    returns is |Y|^2 of the Y it returns."""
    import torch

    import paper_1109_4279_amd as wc
    from paper_1109_4279_amd.autograd import pseudofermion_action
    dims, block, m0, csw = (32, 16, 16, 16), (4, 4, 4, 4), -0.1, 1.0
    Un = gauge(dims)
    phi = synth.gaussian_spinor(dims, seed=synth.FORCE_PHI_SEED)
    kw = dict(tol=1e-12, sap_prec="f64", eo=1)
    U = to_dev(Un).requires_grad_(True)
    S = pseudofermion_action(U, to_dev(phi), block=block, m0=m0, csw=csw, **kw)
    (G,) = torch.autograd.grad(S, U)
    lat = wc.Lattice(to_dev(Un), block=block, m0=m0, csw=csw)
    F, Y, X, st = lat.force(to_dev(phi), **kw)
    assert all(s["status"] == 0 for s in st)
    Y = to_np(Y)
    assert S.item() == pytest.approx(np.vdot(Y, Y).real, rel=1e-12)
    Fg = -0.5 * force.traceless_antihermitian(np.einsum("...ab,...cb->...ac", Un, np.conj(to_np(G))))
    assert rel(Fg, to_np(F)) < 1e-9
