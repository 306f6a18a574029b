"""Element-wise oracle parity of the kernel variants that the full-size workloads run.

Which kernel a call takes depends on its size: the block solvers keep the block operator in
registers only when a launch has at most two work items per CU and reload it in every
phase above that (the 24^3 x 48 x 12-rhs and 32^3 x 64 solves), two right-hand sides can
share a block-solver work-group, and the FP64 D stages each 256-site tile in LDS with up to
four rhs per lane.  Each variant is forced here (context options and rhs tiles) or reached
by a launch of the size that selects it, and compared with the oracle: the block solvers
(Sec. 4: MR on D_Lambda, the even/odd block solver of Table 1) and the Schwarz cycle, and
D_w (abstract, Sec. 4) at the 32^3 x 64 production size of Sec. 6."""
import numpy as np
import pytest

import synth
from oracle import dirac, solvers
from tests.helpers import clover, gauge, lattice, maxrel, oracle_D_slabs, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 3e-3, "bf16": 2e-2}
SAP_TOL = {"f64": 1e-12, "f32": 2e-5, "f16": 5e-3, "bf16": 3e-2}
CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2)),
    ((8, 6, 6, 6), (4, 3, 3, 3)),
    ((8, 8, 8, 8), (4, 4, 4, 4)),
]


def _block_ref(U, A, eta, block, colour, nmr, eo, bc_t=1):
    f = solvers.mr_blocks_eo if eo else solvers.mr_blocks
    return f(U, A, eta, block, colour, nmr, bc_t)


@pytest.mark.parametrize("eo", [0, 1])
@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_block_solver_reloading_operator(dims, block, prec, eo):
    """The block solvers with the operator reloaded in every phase (as at full size), both
    colours and both time boundary conditions."""
    m0, csw = -0.1, 1.0
    for bc_t in (1, -1):
        lat = lattice(dims, block, m0, csw, bc_t)
        lat.set_option("sap_cache", 0)
        U, A = gauge(dims), clover(dims, m0, csw)
        eta = synth.gaussian_spinor(dims, seed=71)
        for colour in (0, 1):
            zw, rw = _block_ref(U, A, eta, block, colour, 4, eo, bc_t)
            z, rho = lat.sap_block_mr(to_dev(eta), colour, 4, prec=prec, eo=bool(eo))
            assert rel(to_np(z), zw) < TOL[prec], (bc_t, colour)
            assert rel(to_np(rho), rw) < TOL[prec], (bc_t, colour)


@pytest.mark.parametrize("eo", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_sap_reloading_operator(prec, eo):
    """Three Schwarz cycles with the operator reloaded in every phase; two rhs."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    lat.set_option("sap_cache", 0)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, nrhs=2, seed=72)
    got = to_np(lat.sap(to_dev(eta), ncy=3, nmr=4, prec=prec, eo=bool(eo)))
    for r in range(2):
        want = solvers.sap(U, A, eta[r], block, nmr=4, ncy=3, eo=bool(eo))
        assert rel(got[r], want) < SAP_TOL[prec]


@pytest.mark.parametrize("eo", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_block_solver_two_rhs_per_workgroup(prec, eo):
    """Two rhs per block-solver work-group (three rhs: one pair and a ragged single), in the
    automatic cache mode and with the operator reloaded; 4^4 blocks, where the plain block
    solver on 16-bit storage stages the block operator in LDS for the pair."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    lat.set_tiles(prec, nr_sap=2, nr_sap_eo=2)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, nrhs=3, seed=73)
    for cache in (-1, 0):
        lat.set_option("sap_cache", cache)
        z, rho = lat.sap_block_mr(to_dev(eta), 1, 4, prec=prec, eo=bool(eo))
        z, rho = to_np(z), to_np(rho)
        for r in range(3):
            zw, rw = _block_ref(U, A, eta[r], block, 1, 4, eo)
            assert rel(z[r], zw) < TOL[prec], (cache, r)
            assert rel(rho[r], rw) < TOL[prec], (cache, r)
    got = to_np(lat.sap(to_dev(eta), ncy=3, nmr=4, prec=prec, eo=bool(eo)))
    for r in range(3):
        want = solvers.sap(U, A, eta[r], block, nmr=4, ncy=3, eo=bool(eo))
        assert rel(got[r], want) < SAP_TOL[prec]


@pytest.mark.parametrize("eo", [0, 1])
def test_block_solver_above_two_items_per_cu(eo):
    """12 rhs on 8^4 with 2^4 blocks: 128 blocks of a colour x 12 rhs = 1536 work items, above
    the 512 at which the automatic mode stops caching the operator (the regime of the
    batched 24^3 x 48 solve); every rhs against the oracle in every reduced precision."""
    dims, block, m0, csw = (8, 8, 8, 8), (2, 2, 2, 2), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, nrhs=12, seed=74)
    ref = [_block_ref(U, A, eta[r], block, 0, 4, eo) for r in range(12)]
    for prec in ("f32", "f16", "bf16"):
        z, rho = lat.sap_block_mr(to_dev(eta), 0, 4, prec=prec, eo=bool(eo))
        z, rho = to_np(z), to_np(rho)
        for r in range(12):
            assert rel(z[r], ref[r][0]) < TOL[prec], (prec, r)
            assert rel(rho[r], ref[r][1]) < TOL[prec], (prec, r)


@pytest.mark.timeout(300)
def test_block_solver_16c32_small_blocks():
    """16^3 x 32 with 2^4 blocks: 4096 blocks of a colour in one launch, operator reloaded
    (the automatic choice at this size), FP32, both block solvers."""
    dims, block, m0, csw = (32, 16, 16, 16), (2, 2, 2, 2), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    eta = synth.gaussian_spinor(dims, seed=75)
    for eo in (0, 1):
        zw, rw = _block_ref(U, A, eta, block, 1, 4, eo)
        z, rho = lat.sap_block_mr(to_dev(eta), 1, 4, prec="f32", eo=bool(eo))
        assert rel(to_np(z), zw) < TOL["f32"]
        assert rel(to_np(rho), rw) < TOL["f32"]


@pytest.mark.parametrize("prec,tiles", [("f64", (1, 2, 3, 4)), ("f32", (2, 4)), ("f16", (2, 4)), ("bf16", (4,))])
def test_dirac_rhs_tiles_on_256_site_tiles(prec, tiles):
    """12 rhs on 4^4 tiles with 1..4 rhs per lane: the FP64 D stages each tile's input in LDS
    (four rhs per lane exceed a work-group's LDS and run unstaged); the reduced precisions
    run with and without staging.  Every rhs against the oracle."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    x = synth.gaussian_spinor(dims, nrhs=12, seed=76)
    want = np.stack([dirac.apply_D(U, A, x[r]) for r in range(12)])
    stages = (-1,) if prec == "f64" else (-1, 1)
    for nr in tiles:
        lat.set_tiles(prec, nr_dirac=nr)
        for stage in stages:
            lat.set_option("dirac_stage", stage)
            got = to_np(lat.apply_D(to_dev(x), prec=prec))
            for r in range(12):
                assert rel(got[r], want[r]) < TOL[prec], (nr, stage, r)
                if prec == "f64":
                    assert maxrel(got[r], want[r]) < 1e-12, (nr, r)


@pytest.mark.timeout(600)
def test_dirac_32c64_matches_oracle_on_slabs():
    """D_w at 32^3 x 64 (Sec. 6's production lattice) in every storage precision against the
    oracle on three time slabs: the first (its halo crosses the periodic time boundary), one
    in the middle and the last."""
    dims, block, m0, csw = (64, 32, 32, 32), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    U = gauge(dims)
    x = synth.gaussian_spinor(dims, seed=77)
    got = {p: to_np(lat.apply_D(to_dev(x), prec=p)) for p in ("f64", "f32", "f16", "bf16")}
    T = 2
    ref = oracle_D_slabs(U, [x], m0, csw, starts=[0, 30, 62], T=T, workers=3)
    for t0, (d,) in ref.items():
        for p, g in got.items():
            assert rel(g[t0:t0 + T], d) < TOL[p], (p, t0)
        assert maxrel(got["f64"][t0:t0 + T], d) < 1e-12, t0
