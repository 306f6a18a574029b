"""GPU solves at the full sizes of the benchmark workloads, each checked by the oracle's
FP64 D_w on sampled right-hand sides (Sec. 4 and 6: SAP-preconditioned FGCR to a true
residual of 1e-10): the 12 spin-colour point sources on 24^3 x 48 in the configuration the
batched benchmark times (FP32 arithmetic on BF16 storage, even/odd block solver, FGCR with
the single-precision recursion of an F32 basis, graph capture) and with FP16 storage and
an FP64 basis, the uneven batch {8^3 x 16, 12^3 x 24, 16^3 x 32} with four Gaussian
right-hand sides each on block shapes chosen by the block-shape autotuner, and the
rhs-tile autotuner."""
import numpy as np
import pytest

import synth
from oracle import dirac
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

M0, CSW = -0.1, 1.0


def _true_res(U, A, x, b):
    return dirac.norm(b - dirac.apply_D(U, A, x)) / dirac.norm(b)


def _valid_block(dims, block):
    vol = int(np.prod(block))
    return vol <= 256 and all(L % b == 0 and (L // b) % 2 == 0 for L, b in zip(dims, block))


@pytest.mark.parametrize("storage,basis", [("bf16", "f32"), ("f16", "f64")])
def test_point_sources_24c48_batched_as_benchmarked(storage, basis):
    dims, block = (48, 24, 24, 24), (4, 4, 4, 4)
    lat = lattice(dims, block, M0, CSW)
    b = synth.point_sources(dims)
    x, st = lat.solve(to_dev(b), nkv=16, ncy=5, nmr=4, tol=1e-10, sap_prec=storage, eo=1, use_graph=1,
                      basis_prec=basis)
    assert all(s["status"] == 0 and s["rel_true_res"] <= 1e-10 for s in st)
    x = to_np(x)
    U, A = gauge(dims), clover(dims, M0, CSW)
    for r in (0, 7, 11):  # the oracle's D_w takes a few seconds per rhs at this size
        res = _true_res(U, A, x[r], b[r])
        assert res <= 1e-10
        assert res == pytest.approx(st[r]["rel_true_res"], rel=1e-3, abs=1e-14)


def test_uneven_batch_on_autotuned_blocks():
    import paper_1109_4279_amd as wc
    specs = [((16, 8, 8, 8), (4, 4, 4, 4)), ((24, 12, 12, 12), (4, 3, 3, 3)), ((32, 16, 16, 16), (4, 4, 4, 4))]
    kw = dict(nkv=16, ncy=5, nmr=4, tol=1e-10, sap_prec="f32", eo=1)
    lats, bs = [], []
    for i, (dims, block) in enumerate(specs):
        lat = lattice(dims, block, M0, CSW, seed=synth.GAUGE_SEED + i)
        tuned = lat.autotune_block(**kw)
        assert _valid_block(dims, tuned), (dims, tuned)
        assert lat.block == tuned
        lats.append(lat)
        bs.append(synth.gaussian_spinor(dims, nrhs=4, seed=synth.RHS_SEED + i))
    xs, st = wc.solve_batch(lats, [to_dev(b) for b in bs], **kw)
    k = 0
    for i, (dims, _) in enumerate(specs):
        U, A = gauge(dims, 0.3, synth.GAUGE_SEED + i), clover(dims, M0, CSW, 0.3, synth.GAUGE_SEED + i)
        x = to_np(xs[i])
        for r in range(4):
            assert st[k]["status"] == 0
            assert _true_res(U, A, x[r], bs[i][r]) <= 1e-10
            k += 1
    # the batch solves each system as its own solve on the same blocks would
    x1, s1 = lats[2].solve(to_dev(bs[2][1]), **kw)
    assert rel(to_np(xs[2])[1], to_np(x1)) < 1e-8
    assert abs(s1[0]["iters"] - st[9]["iters"]) <= 1


def test_rhs_tile_autotuner_keeps_solutions():
    dims, block = (16, 8, 8, 8), (4, 4, 4, 4)
    lat = lattice(dims, block, M0, CSW)
    b = synth.point_sources(dims)
    kw = dict(nkv=16, ncy=5, nmr=4, tol=1e-10, sap_prec="f16", eo=1)
    x0, _ = lat.solve(to_dev(b), **kw)
    nd, nd64, ns, ne = lat.autotune(12, prec="f16")
    assert nd in (1, 2, 3, 4) and nd64 in (1, 2, 3, 4) and ns in (1, 2) and ne in (1, 2)
    x1, st = lat.solve(to_dev(b), **kw)
    assert all(s["status"] == 0 for s in st)
    x1 = to_np(x1)
    assert rel(x1, to_np(x0)) < 1e-8
    U, A = gauge(dims), clover(dims, M0, CSW)
    for r in (2, 9):
        assert _true_res(U, A, x1[r], b[r]) <= 1e-10


def test_fp64_dirac_tile_beyond_the_lds_stage():
    """FP64 D_w with 4 rhs per lane on 4^4 tiles: staging the tile's input would take 200 KB
    of LDS, more than a work-group may hold, so that tile runs unstaged.  The FP64 rhs-tile
    autotuner (which tries 1, 2 and 4 rhs per lane) and an FP64 solve with nr_dirac = 4
    both run, and the solve reaches 1e-10."""
    dims, block = (16, 8, 8, 8), (4, 4, 4, 4)
    lat = lattice(dims, block, M0, CSW)
    b = synth.gaussian_spinor(dims, nrhs=4, seed=61)
    nd, nd64, ns, ne = lat.autotune(4, prec="f64")
    assert nd in (1, 2, 3, 4) and nd == nd64 and ns == 1 and ne == 1
    x, st = lat.solve(to_dev(b), nkv=16, ncy=5, nmr=4, tol=1e-10, sap_prec="f64", nr_dirac=4)
    assert all(s["status"] == 0 for s in st)
    U, A = gauge(dims), clover(dims, M0, CSW)
    x = to_np(x)
    for r in (0, 3):
        assert _true_res(U, A, x[r], b[r]) <= 1e-10


@pytest.mark.timeout(900)
def test_solves_32c64_checked_by_the_oracle():
    """32^3 x 64 (Sec. 6's production lattice): the mixed solves on FP32, FP16 and BF16
    storage (BF16 also with the single-precision recursion of an F32 basis) and an
    independent FP64 reference (the plain MR block solver, tolerance 1e-12,
    a different iteration from the mixed solves' even/odd block solver) all have their true
    residual recomputed with the oracle's D over the whole lattice (time slabs); the mixed
    solutions' error against the reference stays within the condition-number bound."""
    from tests.helpers import oracle_true_res
    dims, block = (64, 32, 32, 32), (4, 4, 4, 4)
    lat = lattice(dims, block, M0, CSW)
    U = gauge(dims)
    b = synth.gaussian_spinor(dims)
    xr, sr = lat.solve(to_dev(b), sap_prec="f64", eo=0, tol=1e-12)
    assert sr[0]["status"] == 0
    xs, st = [to_np(xr)], [sr[0]]
    for sp, qp in (("f32", "f64"), ("f16", "f64"), ("bf16", "f64"), ("bf16", "f32")):
        x, s = lat.solve(to_dev(b), sap_prec=sp, eo=1, tol=1e-10, basis_prec=qp)
        assert s[0]["status"] == 0
        xs.append(to_np(x))
        st.append(s[0])
    res = oracle_true_res(U, M0, CSW, xs, [b] * len(xs), T=4, workers=8)
    assert res[0] <= 1.01e-12
    for r, s in zip(res, st):
        assert r == pytest.approx(s["rel_true_res"], rel=1e-2)
    for x, r in zip(xs[1:], res[1:]):
        assert r <= 1e-10
        # |x - x_ref| / |x_ref| <= cond(D) (tol + tol_ref), cond(D) ~ 1e2 for this operator
        assert rel(x, xs[0]) < 2e-8
