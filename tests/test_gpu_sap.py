"""GPU parity of the block MR half-sweep and of the Schwarz preconditioner against the oracle."""
import numpy as np
import pytest

import synth
from oracle import solvers
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2)),
    ((8, 6, 6, 6), (4, 3, 3, 3)),
    ((8, 8, 8, 8), (4, 4, 4, 4)),
]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("colour", [0, 1])
def test_block_mr_matches_oracle(dims, block, colour):
    m0, csw = -0.1, 1.0
    for bc_t in (1, -1):
        lat = lattice(dims, block, m0, csw, bc_t)
        U, A = gauge(dims), clover(dims, m0, csw)
        eta = synth.gaussian_spinor(dims, seed=31)
        z, rho = lat.sap_block_mr(to_dev(eta), colour, 4, prec="f64")
        zw, rw = solvers.mr_blocks(U, A, eta, block, colour, 4, bc_t)
        assert rel(to_np(z), zw) < 1e-12
        assert rel(to_np(rho), rw) < 1e-12
        z32, r32 = lat.sap_block_mr(to_dev(eta), colour, 4, prec="f32")
        assert rel(to_np(z32), zw) < 1e-5
        assert rel(to_np(r32), rw) < 1e-5


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-5), ("f16", 5e-3), ("bf16", 3e-2)])
def test_sap_matches_oracle(dims, block, prec, tol):
    m0, csw = -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, nrhs=2, seed=32)
    got = to_np(lat.sap(to_dev(eta), ncy=3, nmr=4, prec=prec))
    for r in range(2):
        want = solvers.sap(U, A, eta[r], block, nmr=4, ncy=3)
        assert rel(got[r], want) < tol


def test_sap_nmr_zero_is_identity_on_nothing():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block)
    eta = to_dev(synth.gaussian_spinor(dims, seed=33))
    z, rho = lat.sap_block_mr(eta, 0, 0)
    assert np.abs(to_np(z)).max() == 0.0
