"""GPU FGMRES-DR (Sec. 4): dense-LU parity on 4^4, iteration counts against the oracle,
oracle-checked true residuals with mixed precision, several right-hand sides, graph replay,
and the regime deflation is for (an operator with small eigenvalues)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dense, dirac, solvers
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _true_res(dims, m0, csw, x, b, seed=synth.GAUGE_SEED):
    U = synth.gauge_field(dims, seed=seed)
    A = dirac.clover_matrix(U, m0, csw)
    return dirac.norm(b - dirac.apply_D(U, A, x)) / dirac.norm(b)


@pytest.mark.parametrize("k", [0, 3])
@pytest.mark.parametrize("sap_prec", ["f64", "f32"])
def test_fgmres_dr_4444_matches_dense_lu(sap_prec, k):
    dims, block, m0, csw = (4, 4, 4, 4), (2, 2, 2, 2), 0.0, 1.0
    lat = lattice(dims, block, m0, csw)
    U, A = gauge(dims), clover(dims, m0, csw)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve_fgmres_dr(to_dev(b), k=k, nkv=8, ncy=5, nmr=4, tol=1e-10, sap_prec=sap_prec)
    x = to_np(x)
    assert st[0]["status"] == 0
    assert dirac.norm(b - dirac.apply_D(U, A, x)) / dirac.norm(b) <= 1e-10
    M = dense.assemble(U, A)
    xd = sla.lu_solve(sla.lu_factor(M), b.ravel()).reshape(b.shape)
    assert rel(x, xd) < np.linalg.cond(M) * 1e-10
    if sap_prec == "f64":
        ref = solvers.sap_fgmres_dr(U, A, b, block, nmr=4, ncy=5, m=8, k=k, tol=1e-10)
        assert abs(st[0]["iters"] - ref.iters) <= 1


@pytest.mark.parametrize("sap_prec,eo", [("f32", 0), ("f32", 1), ("f16", 1)])
def test_fgmres_dr_16c32_mixed(sap_prec, eo):
    dims, block, m0, csw = (32, 16, 16, 16), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve_fgmres_dr(to_dev(b), k=8, nkv=16, tol=1e-10, sap_prec=sap_prec, eo=eo)
    assert st[0]["status"] == 0 and st[0]["restarts"] >= 1
    assert _true_res(dims, m0, csw, to_np(x), b) <= 1e-10
    x64, _ = lat.solve(to_dev(b), sap_prec="f64", tol=1e-10)
    assert rel(to_np(x), to_np(x64)) < 1e-8


def test_fgmres_dr_several_rhs_and_graph_replay():
    """Three right-hand sides in one solve (restart 6, 3 deflated vectors: several deflated
    restarts), each reaching the tolerance and matching its single-rhs solve; eager and
    graph-replayed solves agree bitwise."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    b = synth.gaussian_spinor(dims, nrhs=3, seed=61)
    kw = dict(k=3, nkv=6, ncy=2, nmr=2, tol=1e-10, sap_prec="f32")
    xg, sg = lat.solve_fgmres_dr(to_dev(b), use_graph=1, **kw)
    xe, se = lat.solve_fgmres_dr(to_dev(b), use_graph=0, **kw)
    assert np.array_equal(to_np(xg), to_np(xe))
    assert [s["iters"] for s in sg] == [s["iters"] for s in se]
    xg = to_np(xg)
    for r in range(3):
        assert sg[r]["status"] == 0 and sg[r]["restarts"] >= 2
        assert _true_res(dims, m0, csw, xg[r], b[r]) <= 1e-10
        x1, s1 = lat.solve_fgmres_dr(to_dev(b[r]), **kw)
        assert rel(xg[r], to_np(x1)) < 1e-8
        assert abs(s1[0]["iters"] - sg[r]["iters"]) <= 1


def test_fgmres_dr_deflation_helps_near_critical():
    """m0 close to the critical mass of the synthetic field: small eigenvalues slow the
    restarted solvers; keeping 8 harmonic Ritz vectors needs fewer preconditioner calls than
    FGCR and restarted FGMRES with the same 16 vectors."""
    dims, block, m0, csw = (16, 8, 8, 8), (4, 4, 4, 4), -0.17, 1.0  # FGCR needs ~740 steps here
    lat = lattice(dims, block, m0, csw)
    b = synth.gaussian_spinor(dims)
    kw = dict(nkv=16, ncy=2, nmr=2, tol=1e-10, sap_prec="f32", maxit=3000)
    _, s_gcr = lat.solve(to_dev(b), check=False, **kw)
    _, s_gm = lat.solve_fgmres_dr(to_dev(b), k=0, check=False, **kw)
    x, s_dr = lat.solve_fgmres_dr(to_dev(b), k=8, **kw)
    assert s_dr[0]["status"] == 0
    assert _true_res(dims, m0, csw, to_np(x), b) <= 1e-10
    assert s_dr[0]["iters"] < s_gm[0]["iters"]
    assert s_dr[0]["iters"] < s_gcr[0]["iters"]


def test_fgmres_dr_uneven_batch():
    """Lattices of three sizes (one with 4x3x3x3 blocks) and several rhs each in one
    FGMRES-DR solve."""
    import paper_1109_4279_amd as wc
    m0, csw = -0.1, 1.0
    specs = [((16, 8, 8, 8), (4, 4, 4, 4)), ((24, 12, 12, 12), (4, 3, 3, 3)), ((8, 4, 4, 4), (2, 2, 2, 2))]
    lats, bs = [], []
    for i, (dims, block) in enumerate(specs):
        lats.append(lattice(dims, block, m0, csw, seed=synth.GAUGE_SEED + i))
        bs.append(synth.gaussian_spinor(dims, nrhs=2, seed=synth.RHS_SEED + i))
    xs, st = wc.solve_batch(lats, [to_dev(b) for b in bs], tol=1e-10, sap_prec="f32", eo=1, nkv=8, k=3)
    k = 0
    for i, (dims, block) in enumerate(specs):
        x = to_np(xs[i])
        for r in range(2):
            assert st[k]["status"] == 0
            assert _true_res(dims, m0, csw, x[r], bs[i][r], seed=synth.GAUGE_SEED + i) <= 1e-10
            k += 1


def test_fgmres_dr_argument_errors():
    import paper_1109_4279_amd as wc
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block)
    b = to_dev(synth.gaussian_spinor(dims))
    with pytest.raises(wc.WCError) as e:
        lat.solve_fgmres_dr(b, k=8, nkv=8)
    assert e.value.code == -1
    with pytest.raises(wc.WCError):
        lat.solve_fgmres_dr(b, k=-1, nkv=8)
