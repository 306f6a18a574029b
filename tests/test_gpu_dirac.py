"""GPU parity of the clover setup and of D_w / D_Lambda against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import dirac
from tests.helpers import clover, gauge, lattice, maxrel, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

# (dims, block): several tiles, a ragged last work-group (V % 256 != 0), odd block extents
CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2)),
    ((8, 6, 6, 6), (4, 3, 3, 3)),
    ((8, 4, 4, 8), (4, 2, 2, 4)),
    ((6, 4, 2, 4), (3, 2, 1, 2)),
]
TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 3e-3, "bf16": 2e-2}


@pytest.mark.parametrize("dims,block", CASES)
def test_clover_blocks_match_oracle(dims, block):
    m0, csw = -0.1, 1.0
    lat = lattice(dims, block, m0, csw)
    A = to_np(lat.clover())
    ref = clover(dims, m0, csw)
    assert np.abs(A[..., 0, :, :] - ref[..., :6, :6]).max() < 1e-13
    assert np.abs(A[..., 1, :, :] - ref[..., 6:, 6:]).max() < 1e-13


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_dirac_full_matches_oracle(dims, block, prec, bc_t):
    m0, csw = -0.1, 1.0
    lat = lattice(dims, block, m0, csw, bc_t)
    U, A = gauge(dims), clover(dims, m0, csw)
    x = synth.gaussian_spinor(dims, nrhs=3, seed=7)
    got = to_np(lat.apply_D(to_dev(x), prec=prec))
    want = dirac.apply_D(U, A, x, bc_t)
    assert rel(got, want) < TOL[prec]
    if prec == "f64":
        assert maxrel(got, want) < 1e-12


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dirac_blocks_and_dagger_match_oracle(dims, block, prec):
    m0, csw = 0.2, 1.3
    for bc_t in (1, -1):
        lat = lattice(dims, block, m0, csw, bc_t)
        U, A = gauge(dims), clover(dims, m0, csw)
        x = synth.gaussian_spinor(dims, seed=8)
        got = to_np(lat.apply_D(to_dev(x), prec=prec, region="blocks"))
        want = dirac.apply_D(U, A, x, bc_t, block=block)
        assert rel(got, want) < TOL[prec]
        got = to_np(lat.apply_D(to_dev(x), prec=prec, dagger=True))
        want = dirac.apply_Ddag(U, A, x, bc_t)
        assert rel(got, want) < TOL[prec]


@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5, 12])
def test_dirac_multi_rhs_equals_single(nrhs):
    dims, block = (8, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block)
    x = to_dev(synth.gaussian_spinor(dims, nrhs=nrhs, seed=9))
    many = to_np(lat.apply_D(x))
    for r in range(nrhs):
        one = to_np(lat.apply_D(x[r].contiguous()))
        assert np.array_equal(many[r], one)


def test_dirac_full_size_16c32():
    """The benchmark workload (16^3 x 32, 4^4 blocks, m0 = -0.1, c_sw = 1): every output
    element against the oracle, FP64 and FP32."""
    dims, block = (32, 16, 16, 16), (4, 4, 4, 4)
    lat = lattice(dims, block)
    U, A = gauge(dims), clover(dims, -0.1, 1.0)
    x = synth.gaussian_spinor(dims, seed=synth.RHS_SEED)
    want = dirac.apply_D(U, A, x)
    got = to_np(lat.apply_D(to_dev(x), prec="f64"))
    assert maxrel(got, want) < 1e-12
    got = to_np(lat.apply_D(to_dev(x), prec="f32"))
    assert rel(got, want) < 1e-5
    got = to_np(lat.apply_D(to_dev(x), prec="f16"))
    assert rel(got, want) < TOL["f16"]


def test_dirac_gamma5_hermiticity_32c64():
    """At 32^3 x 64 (too large to hold the oracle's clover in a test): <y, D x> = <g5 D g5 y, x>,
    and the FP32 / 16-bit operators agree with the FP64 one within their bounds."""
    import torch
    dims, block = (64, 32, 32, 32), (4, 4, 4, 4)
    lat = lattice(dims, block)
    x = to_dev(synth.gaussian_spinor(dims, seed=1))
    y = to_dev(synth.gaussian_spinor(dims, seed=2))
    Dx = lat.apply_D(x)
    Ddy = lat.apply_D(y, dagger=True)
    lhs = torch.vdot(y.flatten(), Dx.flatten()).item()
    rhs = torch.vdot(Ddy.flatten(), x.flatten()).item()
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    for prec in ("f32", "f16", "bf16"):
        d = lat.apply_D(x, prec=prec)
        assert (torch.linalg.vector_norm(d - Dx) / torch.linalg.vector_norm(Dx)).item() < TOL[prec]


def test_geometry_errors():
    import paper_1109_4279_amd as wc
    U = to_dev(gauge((4, 4, 4, 4)))
    with pytest.raises(wc.WCError) as e:
        wc.Lattice(U, block=(4, 4, 4, 4))  # one block per axis: no chessboard
    assert e.value.code == -2
    with pytest.raises(wc.WCError):
        wc.Lattice(U, block=(3, 2, 2, 2))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_dirac_on_links_outside_su3(prec):
    """Links moved off SU(3) (a random 5 % perturbation; nothing in the storage may assume
    unitarity, e.g. rebuild a row from the other two): D_w and D_Lambda match the oracle on
    the field as given, in every storage precision."""
    import paper_1109_4279_amd as wc
    dims, block, m0, csw = (8, 4, 4, 4), (2, 2, 2, 2), -0.1, 1.0
    rng = np.random.default_rng(17)
    U = synth.gauge_field(dims)
    U = U + 0.05 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    A = dirac.clover_matrix(U, m0, csw)
    lat = wc.Lattice(to_dev(U), block=block, m0=m0, csw=csw)
    x = synth.gaussian_spinor(dims, nrhs=2, seed=9)
    got = to_np(lat.apply_D(to_dev(x), prec=prec))
    assert rel(got, dirac.apply_D(U, A, x)) < TOL[prec]
    got = to_np(lat.apply_D(to_dev(x), prec=prec, region="blocks"))
    assert rel(got, dirac.apply_D(U, A, x, block=block)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_dirac_site_scales_span_wide_ranges(prec):
    """16-bit storage keeps one scale per site and the values relative to it: on a spinor
    whose site norms span 10^-12 .. 10^12 (far outside FP16's 6e-8 .. 65504), every output
    site of D_w is within the storage rounding of the largest site norm in its stencil.
    Without the site scales the small sites flush to zero and the large ones overflow."""
    dims, block = (8, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block)
    U, A = gauge(dims), clover(dims, -0.1, 1.0)
    rng = np.random.default_rng(23)
    x = synth.gaussian_spinor(dims, nrhs=2, seed=10)
    x = x * 10.0 ** rng.uniform(-12, 12, size=x.shape[:5])[..., None, None]
    got = to_np(lat.apply_D(to_dev(x), prec=prec))
    want = dirac.apply_D(U, A, x)
    s = np.linalg.norm(x, axis=(-2, -1))
    m = s.copy()
    for mu in range(4):
        for d in (1, -1):
            m = np.maximum(m, np.roll(s, d, axis=1 + mu))
    err = np.linalg.norm(got - want, axis=(-2, -1))
    assert np.all(err <= 4 * TOL[prec] * m)


def test_binding_checks_tensor_arguments():
    """The Python binding rejects, before the library sees a pointer, tensors the kernels
    would index out of bounds: an output or initial guess of another shape, an output that
    overlaps the input, Y and X of different right-hand-side counts, more than one
    pseudofermion field, and spinors of the wrong rank."""
    import torch
    import paper_1109_4279_amd as wc
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    lat = lattice(dims, block)
    x = to_dev(synth.gaussian_spinor(dims, nrhs=2, seed=3))
    one = x[0].contiguous()
    with pytest.raises(wc.WCError, match="out has shape"):
        lat.apply_D(x, out=lat.new_spinor(1))
    with pytest.raises(wc.WCError, match="overlaps"):
        lat.apply_D(x, out=x)
    with pytest.raises(wc.WCError, match="x0 has shape"):
        lat.solve(x, x0=one)
    with pytest.raises(wc.WCError, match="x0 has shape"):
        lat.solve_fgmres_dr(one, k=2, x0=x)
    with pytest.raises(wc.WCError, match="Y has shape"):
        lat.link_grad(one, x)
    with pytest.raises(wc.WCError, match="phi must be one field"):
        lat.force(x)
    with pytest.raises(wc.WCError, match="must be"):
        lat.apply_D(x.reshape((1,) + tuple(x.shape)))
    with pytest.raises(wc.WCError, match="complex128"):
        lat.apply_D(x.to(torch.complex64))
    U = to_dev(gauge(dims))
    with pytest.raises(wc.WCError, match="U must be"):
        wc.Lattice(U[:3].contiguous(), block=block)
    with pytest.raises(wc.WCError, match="source tensors"):
        wc.solve_batch([lat, lat], [x])
    # a valid caller-provided output is used as given
    out = lat.new_spinor(2)
    assert lat.apply_D(x, out=out) is out
    assert np.array_equal(to_np(out), to_np(lat.apply_D(x)))


def test_clover_constant_flux_closed_form():
    """The library's clover blocks on a constant abelian flux equal the closed form
    (4 + m0) - (c_sw / 2) sin(phi) sigma_{mu nu} (x) diag(1, -1, 0) at every site."""
    import paper_1109_4279_amd as wc
    from tests.test_oracle_operator import _flux_field, clover_flux_closed_form
    dims, block, m0, csw = (8, 8, 4, 8), (4, 4, 2, 4), -0.1, 1.3
    phi = 2 * np.pi * 3 / 8
    for mu, nu in [(0, 1), (0, 3), (1, 3), (3, 2)]:
        lat = wc.Lattice(to_dev(_flux_field(dims, mu, nu, phi)), block=block, m0=m0, csw=csw)
        A = to_np(lat.clover())
        want = clover_flux_closed_form(mu, nu, phi, m0, csw)
        assert np.abs(A[..., 0, :, :] - want[:6, :6]).max() < 1e-14, (mu, nu)
        assert np.abs(A[..., 1, :, :] - want[6:, 6:]).max() < 1e-14, (mu, nu)
