"""GPU parity of the even/odd-preconditioned block solver, of the Schwarz preconditioner built
on it and of FGCR solves that use it, against the oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, solvers
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

# 2^4 and 4^4 blocks; 4x3x3x3 blocks (corner parity varies from block to block); 3^4 blocks
# (odd volume: one lane of the work-group has an even site and no odd one)
CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2)),
    ((8, 6, 6, 6), (4, 3, 3, 3)),
    ((8, 8, 8, 8), (4, 4, 4, 4)),
    ((6, 6, 6, 6), (3, 3, 3, 3)),
]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("colour", [0, 1])
def test_block_mr_eo_matches_oracle(dims, block, colour):
    m0, csw = -0.1, 1.0
    for bc_t in (1, -1):
        lat = lattice(dims, block, m0, csw, bc_t)
        U, A = gauge(dims), clover(dims, m0, csw)
        eta = synth.gaussian_spinor(dims, seed=51)
        zw, rw = solvers.mr_blocks_eo(U, A, eta, block, colour, 4, bc_t)
        z, rho = lat.sap_block_mr(to_dev(eta), colour, 4, prec="f64", eo=True)
        assert rel(to_np(z), zw) < 1e-12
        assert rel(to_np(rho), rw) < 1e-12
        # the block residual on the odd sites is stored as exactly zero
        par = dirac.site_parity(dims)[..., None, None]
        assert np.abs(np.where(par == 1, to_np(rho), 0)).max() == 0.0
        for prec, tol in (("f32", 1e-5), ("f16", 3e-3), ("bf16", 2e-2)):
            zp, rp = lat.sap_block_mr(to_dev(eta), colour, 4, prec=prec, eo=True)
            assert rel(to_np(zp), zw) < tol, prec
            assert rel(to_np(rp), rw) < tol, prec


def test_block_mr_eo_zero_steps():
    """nmr = 0: z_e = 0 and z_o = A_oo^-1 eta_o, the exact odd half of the block solve."""
    dims, block, m0, csw = (4, 4, 4, 4), (2, 2, 2, 2), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, seed=52)
    zw, rw = solvers.mr_blocks_eo(U, A, eta, block, 1, 0)
    z, rho = lat.sap_block_mr(to_dev(eta), 1, 0, prec="f64", eo=True)
    assert rel(to_np(z), zw) < 1e-13
    assert rel(to_np(rho), rw) < 1e-13


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-5), ("f16", 5e-3), ("bf16", 3e-2)])
def test_sap_eo_matches_oracle(dims, block, prec, tol):
    m0, csw = -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, nrhs=2, seed=53)
    got = to_np(lat.sap(to_dev(eta), ncy=3, nmr=4, prec=prec, eo=True))
    for r in range(2):
        want = solvers.sap(U, A, eta[r], block, nmr=4, ncy=3, eo=True)
        assert rel(got[r], want) < tol


@pytest.mark.parametrize("sap_prec", ["f64", "f32", "f16"])
def test_fgcr_eo_4444_matches_dense_lu(sap_prec):
    dims, block, m0, csw = (4, 4, 4, 4), (2, 2, 2, 2), 0.0, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve(to_dev(b), nkv=8, ncy=5, nmr=4, tol=1e-10, sap_prec=sap_prec, eo=1)
    x = to_np(x)
    assert st[0]["status"] == 0
    assert dirac.norm(b - dirac.apply_D(U, A, x)) / dirac.norm(b) <= 1e-10
    M = dense.assemble(U, A)
    xd = sla.lu_solve(sla.lu_factor(M), b.ravel()).reshape(b.shape)
    assert rel(x, xd) < np.linalg.cond(M) * 1e-10
    if sap_prec == "f64":
        ref = solvers.sap_fgcr(U, A, b, block, nmr=4, ncy=5, nkv=8, tol=1e-10, eo=True)
        assert abs(st[0]["iters"] - ref.iters) <= 1


@pytest.mark.parametrize("sap_prec", ["f32", "bf16"])
def test_fgcr_eo_two_rhs_per_workgroup(sap_prec):
    """Two right-hand sides share each block-solver work-group (three rhs: one group of two,
    one ragged group of one).  Every solve reaches the FP64 tolerance and matches the solve
    with one rhs per work-group."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    b = synth.gaussian_spinor(dims, nrhs=3, seed=55)
    x2, st2 = lat.solve(to_dev(b), sap_prec=sap_prec, tol=1e-10, eo=1, nr_sap=2)
    x1, st1 = lat.solve(to_dev(b), sap_prec=sap_prec, tol=1e-10, eo=1, nr_sap=1)
    x2, x1 = to_np(x2), to_np(x1)
    for r in range(3):
        assert st2[r]["status"] == 0
        assert dirac.norm(b[r] - dirac.apply_D(U, A, x2[r])) / dirac.norm(b[r]) <= 1e-10
        assert abs(st2[r]["iters"] - st1[r]["iters"]) <= 1
        assert rel(x2[r], x1[r]) < 1e-8


def test_fgcr_eo_16c32_and_batch():
    import paper_1109_4279_amd as wc
    dims, block, m0, csw = (32, 16, 16, 16), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    b = synth.gaussian_spinor(dims)
    x64, st64 = lat.solve(to_dev(b), sap_prec="f64", tol=1e-10)
    its = {}
    for prec in ("f64", "f32", "f16"):
        x, st = lat.solve(to_dev(b), sap_prec=prec, tol=1e-10, eo=1)
        assert st[0]["status"] == 0
        assert dirac.norm(b - dirac.apply_D(U, A, to_np(x))) / dirac.norm(b) <= 1e-10
        assert rel(to_np(x), to_np(x64)) < 1e-8
        its[prec] = st[0]["iters"]
    # the even/odd block solver is the stronger preconditioner at equal nmr
    assert its["f64"] < st64[0]["iters"]
    # uneven batch of lattices with several right-hand sides each
    specs = [((16, 8, 8, 8), (4, 4, 4, 4)), ((24, 12, 12, 12), (4, 3, 3, 3)), ((8, 4, 4, 4), (2, 2, 2, 2))]
    lats, bs = [], []
    for i, (d, bl) in enumerate(specs):
        lats.append(lattice(d, bl, m0, csw, seed=synth.GAUGE_SEED + i))
        bs.append(synth.gaussian_spinor(d, nrhs=3, seed=synth.RHS_SEED + i))
    xs, st = wc.solve_batch(lats, [to_dev(v) for v in bs], tol=1e-10, sap_prec="f16", eo=1)
    k = 0
    for i, (d, bl) in enumerate(specs):
        Ui = synth.gauge_field(d, seed=synth.GAUGE_SEED + i)
        Ai = dirac.clover_matrix(Ui, m0, csw)
        x = to_np(xs[i])
        for r in range(3):
            assert st[k]["status"] == 0
            assert dirac.norm(bs[i][r] - dirac.apply_D(Ui, Ai, x[r])) / dirac.norm(bs[i][r]) <= 1e-10
            k += 1
