"""FGCR robustness (Sec. 4: restarts): Gram-Schmidt close to the critical mass against the
oracle's iteration counts, the stagnation test, the restart history and phase times, and
graphs that stay valid when another call reallocates the context's work fields."""
import os

import numpy as np
import pytest

import synth
from oracle import dirac
from tests.helpers import clover, gauge, lattice, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fgcr_near_critical_8x8x8x8.txt")


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        head, hist = line.split("|")
        eo, iters, restarts = (int(v) for v in head.split())
        rows[eo] = (iters, restarts, [float(v) for v in hist.split()])
    return rows


@pytest.mark.parametrize("eo", [0, 1])
def test_fgcr_near_critical_matches_oracle_iterations(eo):
    """8^4 at m0 = -0.17 (about 0.01 above the critical mass): the GPU's FP64 SAP-FGCR(16)
    (classical Gram-Schmidt with a second pass wherever the first cancels) takes the
    oracle's iteration count (modified Gram-Schmidt) within one, and its true residual after
    every restart follows the oracle's."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.17, 1.0
    iters, restarts, hist = _golden()[eo]
    lat = lattice(dims, block, m0, csw)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve(to_dev(b), sap_prec="f64", eo=eo, nkv=16, ncy=5, nmr=4, tol=1e-10)
    s = st[0]
    assert s["status"] == 0
    assert abs(s["iters"] - iters) <= 1
    assert s["restarts"] == restarts
    assert s["reorth"] > 0  # close to critical the first pass cancels
    assert s["nhist"] == s["restarts"]
    for got, want in zip(s["res_hist"][:-1], hist[:-1]):
        assert got == pytest.approx(want, rel=0.2)
    U, A = gauge(dims), clover(dims, m0, csw)
    assert dirac.norm(b - dirac.apply_D(U, A, to_np(x))) / dirac.norm(b) <= 1e-10


def test_fgcr_near_critical_f32_basis():
    """The same 8^4 system with the F32 basis: cycles of 16 directions whose first
    Gram-Schmidt pass cancels against F32-stored vectors still take their second pass, and
    the solve reaches 1e-10 by the oracle's D within two iterations of the oracle's FP64
    count."""
    dims, block, m0, csw = (8, 8, 8, 8), (4, 4, 4, 4), -0.17, 1.0
    iters, _restarts, _hist = _golden()[0]
    lat = lattice(dims, block, m0, csw)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve(to_dev(b), sap_prec="f64", eo=0, nkv=16, ncy=5, nmr=4, tol=1e-10, basis_prec="f32")
    s = st[0]
    assert s["status"] == 0
    assert s["reorth"] > 0
    assert abs(s["iters"] - iters) <= 2
    U, A = gauge(dims), clover(dims, m0, csw)
    assert dirac.norm(b - dirac.apply_D(U, A, to_np(x))) / dirac.norm(b) <= 1e-10


def test_stagnation_stops_the_solve():
    """A tolerance below FP64 rounding: the true residual stops dropping, and after `stag`
    restarts without a drop the solve returns WC_ERR_NOT_CONVERGED with x and the stats
    (history included) written, well before maxit."""
    import paper_1109_4279_amd as wc
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block, 0.0, 1.0)
    b = synth.gaussian_spinor(dims)
    x, st = lat.solve(to_dev(b), sap_prec="f64", tol=1e-30, nkv=4, maxit=2000, stag=3, check=False)
    s = st[0]
    assert s["status"] == -5 and s["stagnated"] == 1
    assert s["iters"] < 2000
    h = s["res_hist"]
    assert len(h) == s["restarts"] >= 4
    # each of the last three restarts left the residual no lower than the one before it
    assert all(h[i] >= h[i - 1] for i in range(len(h) - 3, len(h)))
    assert h[-1] < 1e-13
    U, A = gauge(dims), clover(dims, 0.0, 1.0)
    assert dirac.norm(b - dirac.apply_D(U, A, to_np(x))) / dirac.norm(b) < 1e-13
    with pytest.raises(wc.WCError, match="stagnated"):
        lat.solve(to_dev(b), sap_prec="f64", tol=1e-30, nkv=4, maxit=2000, stag=3)
    # stag = 0 switches the test off: the same solve runs to maxit
    _, st0 = lat.solve(to_dev(b), sap_prec="f64", tol=1e-30, nkv=4, maxit=120, stag=0, check=False)
    assert st0[0]["stagnated"] == 0 and st0[0]["iters"] == 120


def test_phase_times_and_history():
    """timing = 1 runs the cycles eagerly with events between phases: the solution is the
    graph-replayed one bit for bit, and the phase times add up to the cycles' time."""
    dims, block = (16, 8, 8, 8), (4, 4, 4, 4)
    lat = lattice(dims, block)
    b = to_dev(synth.gaussian_spinor(dims, seed=81))
    x0, s0 = lat.solve(b, sap_prec="f32", eo=1, tol=1e-10)
    x1, s1 = lat.solve(b, sap_prec="f32", eo=1, tol=1e-10, timing=1)
    assert np.array_equal(to_np(x0), to_np(x1))
    t = s1[0]
    assert t["timed"] == 1 and s0[0]["timed"] == 0
    parts = t["t_sap_ms"] + t["t_dirac_ms"] + t["t_blas_ms"]
    assert t["t_sap_ms"] > t["t_dirac_ms"] > 0 and t["t_blas_ms"] > 0
    # the cycles' span also holds the host's read of the residuals between restarts
    assert 0.5 * t["t_cycles_ms"] < parts <= 1.001 * t["t_cycles_ms"]
    assert t["t_setup_ms"] > 0 and t["t_setup_ms"] + t["t_cycles_ms"] <= t["time_ms"] * 1.001
    assert t["nhist"] == t["restarts"] and t["res_hist"][-1] == pytest.approx(t["rel_true_res"], rel=1e-12)


@pytest.mark.parametrize("k", [None, 3])
def test_graph_survives_reallocated_fields(k):
    """A solve captures its cycle as a graph over the context's Schwarz fields; a call in a
    wider precision (an FP64 Schwarz application, an FP32 solve) reallocates those fields.
    Solving again in the first precision must recapture, not replay over freed memory: the
    result equals the first solve bit for bit."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    lat = lattice(dims, block)
    b = to_dev(synth.gaussian_spinor(dims, seed=82))

    def solve(prec):
        if k is None:
            return lat.solve(b, sap_prec=prec, eo=1, tol=1e-10)
        return lat.solve_fgmres_dr(b, k=k, nkv=12, sap_prec=prec, eo=1, tol=1e-10)

    x0, s0 = solve("f16")
    lat.sap(b, ncy=2, nmr=2, prec="f64", eo=True)
    x1, s1 = solve("f16")
    solve("f32")
    x2, s2 = solve("f16")
    assert np.array_equal(to_np(x0), to_np(x1))
    assert np.array_equal(to_np(x0), to_np(x2))
    assert s0[0]["iters"] == s1[0]["iters"] == s2[0]["iters"]


def test_options_and_tiles_errors():
    import paper_1109_4279_amd as wc
    lat = lattice((4, 4, 4, 4), (2, 2, 2, 2))
    with pytest.raises(KeyError):
        lat.set_option("nope", 0)
    with pytest.raises(wc.WCError):
        lat.set_option("sap_cache", 2)
    with pytest.raises(wc.WCError):
        lat.set_tiles("f64", nr_sap=2)
    with pytest.raises(wc.WCError):
        lat.set_tiles("f32", nr_dirac=5)
    lat.set_tiles("f32", 4, 2, 2)
    lat.set_tiles("f32")
