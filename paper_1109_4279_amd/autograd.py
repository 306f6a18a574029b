"""torch.autograd.Functions around the library's operator, solve and pseudofermion action.

Every application of D, D^dag, D^-1 and D^-dag, the action's value, its derivatives and
every link derivative run in libwc; these classes only route tensors:

* ``dirac_apply(U, x)``  y = D[U] x;  backward: dx = D^dag dy = g5 D g5 dy,
  dU = link derivative of Re<dy, D x> (torch's conjugate-gradient convention).
* ``dirac_solve(U, b)``  x = D[U]^-1 b;  backward: db = D^-dag dx (one more solve),
  dU = -(link derivative of Re<db, D x>).
* ``pseudofermion_action(U, phi)``  S = phi^dag (D^dag D)^-1 phi = |Y|^2, Y = D^-dag phi;
  backward: dphi = 2 X with X = D^-1 Y, dU = -2 (link derivative of Re<Y, D X>)
  (dS = -2 Re<Y, dD X>, the HMC fermion force of arXiv:1109.4279 Sec. 1).

Each forward builds a context from the U it is given, so U may itself be a leaf that
autograd differentiates.  Spinors are complex128 [..][L0..L3][4][3] CUDA tensors.
"""
from __future__ import annotations

import torch

from . import Lattice, _params


def _lattice(U, opts):
    return Lattice(U.detach().contiguous(), block=opts["block"], m0=opts["m0"], csw=opts["csw"], bc_t=opts["bc_t"])


def _opts(block, m0, csw, bc_t):
    return {"block": tuple(block), "m0": float(m0), "csw": float(csw), "bc_t": int(bc_t)}


def _adjoint(params):
    """A copy of the solver parameters that solves D^dag x = b."""
    if params.dagger:
        raise ValueError("the autograd functions solve with D; pass params with dagger = 0")
    q = type(params).from_buffer_copy(params)
    q.dagger = 1
    return q


class DiracApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, x, opts):
        lat = _lattice(U, opts)
        xc = x.detach().contiguous()
        ctx.lat = lat
        ctx.save_for_backward(xc)
        return lat.apply_D(xc)

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        lat = ctx.lat
        gy = gy.contiguous()
        gU = lat.link_grad(gy, x) if ctx.needs_input_grad[0] else None
        gx = lat.apply_D(gy, dagger=True) if ctx.needs_input_grad[1] else None
        return gU, gx, None


class DiracSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, b, opts, params):
        adj = _adjoint(params)
        lat = _lattice(U, opts)
        x, _ = lat.solve(b.detach().contiguous(), params=params)
        ctx.lat, ctx.adj = lat, adj
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lat = ctx.lat
        gb, _ = lat.solve(gx.contiguous(), params=ctx.adj)  # db = D^-dag gx
        gU = lat.link_grad(gb, x, coef=-1.0) if ctx.needs_input_grad[0] else None
        return gU, (gb if ctx.needs_input_grad[1] else None), None, None


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, opts, params):
        _adjoint(params)
        lat = _lattice(U, opts)
        S, Y, X, _ = lat.action(phi.detach().contiguous(), params=params)  # Y = D^-dag phi, X = D^-1 Y
        ctx.lat = lat
        ctx.save_for_backward(Y, X)
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gS):
        Y, X = ctx.saved_tensors
        lat = ctx.lat
        g = float(gS)
        gU = lat.link_grad(Y, X, coef=-2.0 * g) if ctx.needs_input_grad[0] else None
        gphi = lat.scale(X, 2.0 * g) if ctx.needs_input_grad[1] else None
        return gU, gphi, None, None


def dirac_apply(U, x, block=(4, 4, 4, 4), m0=0.0, csw=1.0, bc_t=1):
    return DiracApply.apply(U, x, _opts(block, m0, csw, bc_t))


def dirac_solve(U, b, block=(4, 4, 4, 4), m0=0.0, csw=1.0, bc_t=1, params=None, **kw):
    p = _params(params, kw)
    return DiracSolve.apply(U, b, _opts(block, m0, csw, bc_t), p)


def pseudofermion_action(U, phi, block=(4, 4, 4, 4), m0=0.0, csw=1.0, bc_t=1, params=None, **kw):
    p = _params(params, kw)
    return PseudofermionAction.apply(U, phi, _opts(block, m0, csw, bc_t), p)
