"""The quenched-ensemble workload generator (synth.quenched), pinned by what the mathematics
fixes: the SU(2) heatbath's conditional density (mean and second moment by quadrature, and
the closed form I_2/I_1 of the mean), the invariance of the action under overrelaxation,
SU(3) to rounding, the staple against the plaquettes it stands for, the leading terms of the
strong-coupling expansion of the plaquette, and the well-known plaquette of the Wilson
action at beta = 6.0."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, special

from synth import quenched as q


@pytest.mark.parametrize("alpha", [0.3, 1.5, 2.0, 6.0, 20.0])
def test_su2_sampler_matches_its_density(alpha):
    """y0 ~ sqrt(1 - y^2) exp(alpha y): mean and second moment against quadrature of the
    density, the mean also against the closed form I_2(alpha) / I_1(alpha)."""
    g = torch.Generator()
    g.manual_seed(11)
    n = 200_000
    y = q.sample_y0(torch.full((n,), alpha, dtype=torch.float64), g).numpy()
    assert np.all(np.abs(y) <= 1.0)
    w = lambda t: math.sqrt(1 - t * t) * math.exp(alpha * (t - 1))  # noqa: E731
    z = integrate.quad(w, -1, 1)[0]
    m1 = integrate.quad(lambda t: t * w(t), -1, 1)[0] / z
    m2 = integrate.quad(lambda t: t * t * w(t), -1, 1)[0] / z
    assert m1 == pytest.approx(special.iv(2, alpha) / special.iv(1, alpha), rel=1e-8)
    sd1 = math.sqrt(max(m2 - m1 * m1, 1e-12) / n)
    sd2 = math.sqrt(max(np.var(y * y), 1e-12) / n)
    assert abs(y.mean() - m1) < 5 * sd1
    assert abs((y * y).mean() - m2) < 5 * sd2


def test_su2_projection():
    """k V with V in SU(2) and Re tr(r w) = k Re tr(r V) for random r in SU(2)."""
    g = torch.Generator()
    g.manual_seed(3)
    w = torch.complex(torch.randn(50, 2, 2, generator=g, dtype=torch.float64),
                      torch.randn(50, 2, 2, generator=g, dtype=torch.float64))
    k, V = q.su2_project(w)
    eye = torch.eye(2, dtype=w.dtype)
    assert torch.allclose(V @ V.conj().transpose(-1, -2), eye.expand(50, 2, 2), atol=1e-13)
    assert torch.allclose(torch.linalg.det(V), torch.ones(50, dtype=w.dtype), atol=1e-13)
    qv = torch.randn(50, 4, generator=g, dtype=torch.float64)
    r = q._su2_from_quaternion(qv / qv.norm(dim=-1, keepdim=True))
    lhs = torch.diagonal(r @ w, dim1=-2, dim2=-1).sum(-1).real
    rhs = k * torch.diagonal(r @ V, dim1=-2, dim2=-1).sum(-1).real
    assert torch.allclose(lhs, rhs, atol=1e-12)


def _hot(dims, seed):
    g = torch.Generator()
    g.manual_seed(seed)
    z = torch.complex(torch.randn((4,) + dims + (3, 3), generator=g, dtype=torch.float64),
                      torch.randn((4,) + dims + (3, 3), generator=g, dtype=torch.float64))
    return q.reunitarise(z)


def test_staple_sums_the_plaquettes():
    """sum_x Re tr(U_mu(x) A_mu(x)) counts each (mu, nu) plaquette twice per nu != mu:
    sum over mu of it is 4 x the sum of Re tr over all 6 V plaquettes."""
    dims = (4, 3, 4, 2)
    U = _hot(dims, 5)
    tot = sum(float(torch.diagonal(U[mu] @ q.staple(U, mu), dim1=-2, dim2=-1).sum(-1).real.sum()) for mu in range(4))
    vol = math.prod(dims)
    assert tot == pytest.approx(4 * 3 * 6 * vol * q.plaquette(U), rel=1e-12)


def test_overrelaxation_keeps_the_action_and_heatbath_keeps_su3():
    U = _hot((4, 4, 4, 4), 7)
    g = torch.Generator()
    g.manual_seed(9)
    U0 = U.clone()
    s0 = q.action(U, 6.0)
    q.sweep(U, 6.0, g, heatbath=False)
    assert float((U - U0).abs().max()) > 0.1
    assert q.action(U, 6.0) == pytest.approx(s0, rel=1e-12)
    q.sweep(U, 6.0, g, heatbath=True)
    eye = torch.eye(3, dtype=U.dtype)
    assert float((U @ U.conj().transpose(-1, -2) - eye).abs().max()) < 1e-12
    assert float((torch.linalg.det(U) - 1).abs().max()) < 1e-12


def test_strong_coupling_plaquette():
    """Small beta: <Re tr U_p / 3> = beta/18 + beta^2/216 + O(beta^3) for SU(3) (from the
    Haar moments <(Re tr U)^2> = 1/2 and <(Re tr U)^3> = 1/4); a slip in the heatbath's
    coupling (alpha = 2 beta k / 3) would move it by a factor."""
    beta = 0.6
    dims = (4, 4, 4, 4)
    hist = []
    q.ensemble(dims, beta=beta, ntherm=110, nor=0, seed=13, history=hist)
    meas = np.array(hist[10:])
    want = beta / 18 + beta ** 2 / 216
    err = meas.std() / math.sqrt(len(meas))  # heatbath sweeps at small beta are close to independent
    assert abs(meas.mean() - want) < 4 * err + 1e-3  # 1e-3 for the beta^3 terms


def test_beta6_plaquette():
    """beta = 6.0: the Wilson-action plaquette 0.5937 of the quenched SU(3) literature, on
    8^4 from a cold start (16 compound sweeps to thermalise, 20 measured; the tolerance holds
    the statistical error, about 4e-4, and the small-volume shift)."""
    hist = []
    q.ensemble((8, 8, 8, 8), beta=6.0, ntherm=36, nor=2, seed=17, history=hist)
    assert abs(np.mean(hist[16:]) - 0.5937) < 0.0025
