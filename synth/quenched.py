"""Seeded quenched SU(3) gauge ensembles: the self-generated workload of the near-critical
stress runs (Sec. 4 and Fig. 1 of arXiv:1109.4279 study the solvers close to the critical
quark mass on dynamical ensembles, which are not available here).

A workload generator, not part of the method: it samples gauge fields with the weight
exp(-S_W) of the Wilson plaquette action

    S_W = beta * sum_p (1 - Re tr U_p / 3),

and touches none of the solver's arithmetic (no Dirac operator, clover term, Krylov or
Schwarz step).  It runs on torch tensors, on the CPU for the tests and on the GPU for the
benchmark; the same seed gives the same field on one device type.

Algorithm (standard, written from the published methods):
* links are updated one direction and one site parity at a time (the links U_mu(x) of one
  parity do not appear in each other's staples);
* each link gets a Cabibbo-Marinari update (N. Cabibbo and E. Marinari, Phys. Lett. B 119
  (1982) 387): left multiplication by an SU(2) matrix in each of the three subgroups (0,1),
  (0,2), (1,2) in turn, drawn from its exact conditional distribution (heatbath) or
  reflected so that the action does not change (overrelaxation, M. Creutz, Phys. Rev. D 36
  (1987) 515);
* the heatbath's SU(2) element y = y0 + i y.sigma has density proportional to
  sqrt(1 - y0^2) exp(alpha y0) in y0 and a uniform direction of y; y0 is drawn by the
  method of A. D. Kennedy and B. J. Pendleton (Phys. Lett. B 156 (1985) 393) for
  alpha >= 2 and by M. Creutz's (Phys. Rev. D 21 (1980) 2308) below;
* after every sweep the links are projected back onto SU(3).

Conventions as in the package: U[mu][L0][L1][L2][L3][3][3], U[mu] at x the link from x to
x + mu_hat, periodic in every direction.
"""
from __future__ import annotations

import math

import torch

QUENCHED_SEED = 2468
SUBGROUPS = ((0, 1), (0, 2), (1, 2))


def _mm(a, b):
    return torch.matmul(a, b)


def _dag(a):
    return a.conj().transpose(-1, -2)


def staple(U, mu):
    """A_mu(x), the sum over nu != mu of the two staples, so that the plaquettes through
    U_mu(x) are U_mu(x) A_mu(x) (six terms, their Re tr summed by the action)."""
    dims = U.shape[1:5]
    A = torch.zeros(dims + (3, 3), dtype=U.dtype, device=U.device)
    ax_mu = mu
    for nu in range(4):
        if nu == mu:
            continue
        Unu_xmu = torch.roll(U[nu], -1, dims=ax_mu)          # U_nu(x + mu)
        Umu_xnu = torch.roll(U[mu], -1, dims=nu)             # U_mu(x + nu)
        A = A + _mm(_mm(Unu_xmu, _dag(Umu_xnu)), _dag(U[nu]))
        # backward: U_nu(x + mu - nu)^dag U_mu(x - nu)^dag U_nu(x - nu)
        Unu_xmu_mnu = torch.roll(Unu_xmu, 1, dims=nu)
        Umu_mnu = torch.roll(U[mu], 1, dims=nu)
        Unu_mnu = torch.roll(U[nu], 1, dims=nu)
        A = A + _mm(_mm(_dag(Unu_xmu_mnu), _dag(Umu_mnu)), Unu_mnu)
    return A


def plaquette(U) -> float:
    """Mean of Re tr U_p / 3 over the 6 V plaquettes."""
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            p = _mm(_mm(U[mu], torch.roll(U[nu], -1, dims=mu)), _mm(_dag(torch.roll(U[mu], -1, dims=nu)), _dag(U[nu])))
            tot += float(torch.diagonal(p, dim1=-2, dim2=-1).sum(-1).real.mean())
    return tot / (6 * 3)


def action(U, beta: float) -> float:
    """S_W = beta * sum_p (1 - Re tr U_p / 3)."""
    vol = math.prod(U.shape[1:5])
    return beta * 6 * vol * (1.0 - plaquette(U))


def reunitarise(m):
    """Rows Gram-Schmidt orthonormalised, third row conj(row0 x row1): SU(3) to rounding."""
    r0 = m[..., 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = m[..., 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def _uniform_open(n, gen, device):
    """n uniform numbers in (0, 1]."""
    return 1.0 - torch.rand(n, generator=gen, device=device, dtype=torch.float64)


def sample_y0(alpha, gen):
    """y0 in [-1, 1] with density proportional to sqrt(1 - y0^2) exp(alpha y0), one per
    entry of alpha (> 0): Kennedy-Pendleton for alpha >= 2, Creutz's method below."""
    dev = alpha.device
    n = alpha.numel()
    y0 = torch.empty(n, dtype=torch.float64, device=dev)
    todo = torch.arange(n, device=dev)
    while todo.numel():
        a = alpha[todo]
        m = todo.numel()
        big = a >= 2.0
        # Kennedy-Pendleton: x = -(ln r1 + cos^2(2 pi r2) ln r3) / alpha, accept if r4^2 <= 1 - x/2
        r1, r2, r3, r4 = (_uniform_open(m, gen, dev) for _ in range(4))
        x = -(torch.log(r1) + torch.cos(2.0 * math.pi * r2) ** 2 * torch.log(r3)) / a
        kp = 1.0 - x
        kp_ok = r4 * r4 <= 1.0 - 0.5 * x
        # Creutz: exp(alpha y0) uniform on [exp(-alpha), exp(alpha)], accept with sqrt(1 - y0^2)
        u, v = _uniform_open(m, gen, dev), _uniform_open(m, gen, dev)
        cr = 1.0 + torch.log1p(-(1.0 - u) * (-torch.expm1(-2.0 * a))) / a
        cr = cr.clamp(-1.0, 1.0)
        cr_ok = v <= torch.sqrt(1.0 - cr * cr)
        val = torch.where(big, kp, cr)
        ok = torch.where(big, kp_ok, cr_ok)
        y0[todo[ok]] = val[ok]
        todo = todo[~ok]
    return y0


def _su2_from_quaternion(q):
    """[[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]] for q (..., 4)."""
    q0, q1, q2, q3 = q.unbind(-1)
    row0 = torch.stack([torch.complex(q0, q3), torch.complex(q2, q1)], dim=-1)
    row1 = torch.stack([torch.complex(-q2, q1), torch.complex(q0, -q3)], dim=-1)
    return torch.stack([row0, row1], dim=-2)


def su2_project(w):
    """The SU(2)-proportional part of 2x2 matrices w: (k, V) with k >= 0 and V in SU(2),
    k V = [[a, b], [-conj b, conj a]], a = (w00 + conj w11)/2, b = (w01 - conj w10)/2;
    Re tr(r w) = k Re tr(r V) for every r in SU(2)."""
    a = 0.5 * (w[..., 0, 0] + w[..., 1, 1].conj())
    b = 0.5 * (w[..., 0, 1] - w[..., 1, 0].conj())
    k = torch.sqrt(a.real ** 2 + a.imag ** 2 + b.real ** 2 + b.imag ** 2)
    ks = torch.clamp(k, min=1e-300)
    q = torch.stack([a.real / ks, b.imag / ks, b.real / ks, a.imag / ks], dim=-1)
    return k, _su2_from_quaternion(q)


def _embed_left(U, r, i, j):
    """R U with R the identity except rows/columns (i, j) = r (2x2)."""
    out = U.clone()
    ui, uj = U[..., i, :], U[..., j, :]
    out[..., i, :] = r[..., 0, 0, None] * ui + r[..., 0, 1, None] * uj
    out[..., j, :] = r[..., 1, 0, None] * ui + r[..., 1, 1, None] * uj
    return out


def cm_update(Ul, A, beta: float, gen, heatbath: bool):
    """One Cabibbo-Marinari pass over the three SU(2) subgroups of the links Ul (n, 3, 3)
    with staples A (n, 3, 3): heatbath (new element from exp(beta/3 Re tr(U A))) or
    overrelaxation (reflection keeping Re tr(U A))."""
    for (i, j) in SUBGROUPS:
        W = _mm(Ul, A)
        w = W[..., [i, j], :][..., :, [i, j]]
        k, V = su2_project(w)
        if heatbath:
            alpha = (2.0 * beta / 3.0) * k
            y0 = sample_y0(torch.clamp(alpha, min=1e-12), gen)
            n = y0.numel()
            # uniform direction on the sphere: cos(theta) uniform in [-1, 1], phi in [0, 2 pi)
            ct = 2.0 * torch.rand(n, generator=gen, device=Ul.device, dtype=torch.float64) - 1.0
            ph = 2.0 * math.pi * torch.rand(n, generator=gen, device=Ul.device, dtype=torch.float64)
            st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
            rad = torch.sqrt(torch.clamp(1.0 - y0 * y0, min=0.0))
            y = _su2_from_quaternion(torch.stack([y0, rad * st * torch.cos(ph), rad * st * torch.sin(ph), rad * ct], -1))
            r = _mm(y, _dag(V))
        else:
            r = _mm(_dag(V), _dag(V))
        Ul = _embed_left(Ul, r, i, j)
    return Ul


def parity_mask(dims, device):
    c = [torch.arange(d, device=device) for d in dims]
    g = torch.meshgrid(*c, indexing="ij")
    return (g[0] + g[1] + g[2] + g[3]) % 2


def sweep(U, beta: float, gen, heatbath: bool = True):
    """One sweep: every direction, each site parity in turn, one Cabibbo-Marinari update."""
    dims = tuple(U.shape[1:5])
    par = parity_mask(dims, U.device)
    for mu in range(4):
        for p in (0, 1):
            A = staple(U, mu)
            m = par == p
            U[mu][m] = cm_update(U[mu][m], A[m], beta, gen, heatbath)
    return U


def cold_start(dims, device="cpu"):
    U = torch.zeros((4,) + tuple(dims) + (3, 3), dtype=torch.complex128, device=device)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def ensemble(dims, beta: float = 6.0, ntherm: int = 100, nor: int = 4, seed: int = QUENCHED_SEED,
             device="cpu", U=None, history: list | None = None):
    """A thermalised quenched field: from a cold start (or U), ntherm compound sweeps of one
    heatbath and nor overrelaxation sweeps, projected onto SU(3) after each; the plaquette
    after every compound sweep is appended to `history` when given."""
    dims = tuple(int(d) for d in dims)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    U = cold_start(dims, device) if U is None else U.clone()
    for _ in range(ntherm):
        sweep(U, beta, gen, True)
        for _ in range(nor):
            sweep(U, beta, gen, False)
        U = reunitarise(U)
        if history is not None:
            history.append(plaquette(U))
    return U
