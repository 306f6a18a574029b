"""MI355X-native Wilson-clover SAP-FGCR hot path (arXiv:1109.4279) behind a C interface.

Python holds device memory (torch tensors) and marshals arguments; every step of the
operator, the Schwarz preconditioner, the Krylov solver and the force runs in the HIP
library ``libwc.so`` (see ``include/wc.h``).  Importing this package does not load the
library; the first call does, and raises if it has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import PREC, REGION, SolverParams, SolverStats, WCError  # noqa: F401

__all__ = ["Lattice", "SolverParams", "SolverStats", "WCError", "default_params", "solve_batch", "PREC"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, shape_tail=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise WCError(-1, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex128:
        raise WCError(-1, f"{name} must be complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise WCError(-1, f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise WCError(-1, f"{name} has shape {tuple(t.shape)}, expected (..., {shape_tail})")
    return t


def _set_fields(p, kw):
    names = {f[0] for f in SolverParams._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver parameter {k!r} (fields: {', '.join(sorted(names))})")
        if k in ("sap_prec", "basis_prec") and isinstance(v, str):
            v = PREC[v]
        setattr(p, k, v)


def _overlap(a, b):
    pa, pb = a.data_ptr(), b.data_ptr()
    return pa < pb + b.numel() * b.element_size() and pb < pa + a.numel() * a.element_size()


def _params(params, kw):
    """A copy of the caller's parameters (the solve sets x0_given on its copy), or the
    defaults, with the fields named in kw replaced."""
    if params is None:
        return default_params(**kw)
    p = SolverParams.from_buffer_copy(params)
    _set_fields(p, kw)
    return p


def default_params(**kw) -> SolverParams:
    """The library's defaults (wc_default_params) with the fields named in kw replaced;
    sap_prec and basis_prec may be given by name ("f64", "f32", "f16", "bf16")."""
    p = SolverParams()
    _lib.load().wc_default_params(ctypes.byref(p))
    _set_fields(p, kw)
    return p


class Lattice:
    """One lattice: gauge field, clover term and the library context that owns their copies.

    U: complex128 CUDA tensor [4][L0][L1][L2][L3][3][3]; block: Schwarz block shape."""

    def __init__(self, U, block=(4, 4, 4, 4), m0: float = 0.0, csw: float = 1.0, bc_t: int = 1, stream=None):
        lib = _lib.load()
        _need(U, "U", (3, 3))
        if U.dim() != 7 or U.shape[0] != 4:
            raise WCError(-1, f"U must be [4][L0][L1][L2][L3][3][3], got {tuple(U.shape)}")
        self.dims = tuple(int(d) for d in U.shape[1:5])
        self.block = tuple(int(b) for b in block)
        self.m0, self.csw, self.bc_t = float(m0), float(csw), int(bc_t)
        self._U = U
        self._ctx = ctypes.c_void_p()
        dims = (ctypes.c_int * 4)(*self.dims)
        blk = (ctypes.c_int * 4)(*self.block)
        _lib.check(lib.wc_create_gauge(ctypes.byref(self._ctx), dims, blk, _ptr(U), self.bc_t, _stream(stream)))
        _lib.check(lib.wc_create_clover(self._ctx, self.m0, self.csw, _stream(stream)))

    @property
    def volume(self) -> int:
        v = 1
        for d in self.dims:
            v *= d
        return v

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                _lib.load().wc_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    # ------------------------------------------------------------------ helpers
    def _spinor(self, t, name, like=None):
        """Number of right-hand sides of a spinor argument: a complex128 tensor
        [L0..L3][4][3] (one) or [nrhs][L0..L3][4][3] on the lattice's device; with `like`,
        it must have like's shape.  Checked before the library sees the pointer."""
        _need(t, name, self.dims + (4, 3))
        if t.dim() not in (6, 7):
            raise WCError(-1, f"{name} must be [L0..L3][4][3] or [nrhs][L0..L3][4][3], got {tuple(t.shape)}")
        if t.device != self._U.device:
            raise WCError(-1, f"{name} is on {t.device}, the lattice on {self._U.device}")
        if like is not None and t.shape != like.shape:
            raise WCError(-1, f"{name} has shape {tuple(t.shape)}, expected {tuple(like.shape)}")
        return 1 if t.dim() == 6 else int(t.shape[0])

    def new_spinor(self, nrhs=None):
        torch = _torch()
        shape = self.dims + (4, 3) if nrhs is None else (nrhs,) + self.dims + (4, 3)
        return torch.empty(shape, dtype=torch.complex128, device=self._U.device)

    # ------------------------------------------------------------------ operator
    def apply_D(self, x, prec="f64", region="full", dagger=False, out=None, stream=None):
        nrhs = self._spinor(x, "x")
        if out is None:
            out = self.new_spinor(None if x.dim() == 6 else nrhs)
        else:
            self._spinor(out, "out", like=x)
            if _overlap(out, x):
                raise WCError(-1, "out overlaps x")
        _lib.check(_lib.load().wc_apply_D(self._ctx, _ptr(out), _ptr(x), nrhs, PREC[prec], REGION[region],
                                          int(bool(dagger)), _stream(stream)))
        return out

    def clover(self, stream=None):
        torch = _torch()
        A = torch.empty(self.dims + (2, 6, 6), dtype=torch.complex128, device=self._U.device)
        _lib.check(_lib.load().wc_clover_export(self._ctx, _ptr(A), _stream(stream)))
        return A

    def sap_block_mr(self, rho, colour, nmr, prec="f64", eo=False, stream=None):
        """One half-sweep: returns (z, rho_new) as the library computes them (rho is not modified).
        eo selects the even/odd-preconditioned block solver."""
        nrhs = self._spinor(rho, "rho")
        r = rho.clone()
        z = self.new_spinor(None if rho.dim() == 6 else nrhs)
        _lib.check(_lib.load().wc_sap_block_mr(self._ctx, _ptr(z), _ptr(r), nrhs, int(colour), int(nmr), PREC[prec],
                                               int(bool(eo)), _stream(stream)))
        return z, r

    def sap(self, eta, ncy=5, nmr=4, prec="f64", eo=False, stream=None):
        nrhs = self._spinor(eta, "eta")
        psi = self.new_spinor(None if eta.dim() == 6 else nrhs)
        _lib.check(_lib.load().wc_sap(self._ctx, _ptr(psi), _ptr(eta), nrhs, int(ncy), int(nmr), PREC[prec],
                                      int(bool(eo)), _stream(stream)))
        return psi

    def solve(self, b, params: SolverParams | None = None, x0=None, stream=None, check=True, **kw):
        """x = D^-1 b by SAP-preconditioned FGCR.  Returns (x, list of per-rhs stats dicts).
        Solver parameters come from `params` or the keywords (wc_solver_params' fields), e.g.
        sap_prec="bf16", eo=1, and basis_prec="f32" for the single-precision recursion
        between FP64 restarts (cycles then also end at a drop of the residual, 1e-6 unless
        `drop` is given)."""
        nrhs = self._spinor(b, "b")
        p = _params(params, kw)
        if x0 is not None:
            self._spinor(x0, "x0", like=b)
            x = x0.clone()
            p.x0_given = 1
        else:
            x = self.new_spinor(None if b.dim() == 6 else nrhs)
            p.x0_given = 0
        st = (SolverStats * nrhs)()
        rc = _lib.load().wc_fgcr_solve(self._ctx, _ptr(x), _ptr(b), nrhs, ctypes.byref(p), st, _stream(stream))
        stats = [s.as_dict() for s in st]
        if check:
            _lib.check(rc)
        return x, stats

    def solve_fgmres_dr(self, b, k=8, params: SolverParams | None = None, x0=None, stream=None, check=True, **kw):
        """x = D^-1 b by SAP-preconditioned FGMRES-DR: cycles of params.nkv Arnoldi steps, k
        harmonic Ritz vectors kept at every restart (k = 0: restarted FGMRES).  Returns
        (x, list of per-rhs stats dicts)."""
        nrhs = self._spinor(b, "b")
        p = _params(params, kw)
        if x0 is not None:
            self._spinor(x0, "x0", like=b)
            x = x0.clone()
            p.x0_given = 1
        else:
            x = self.new_spinor(None if b.dim() == 6 else nrhs)
            p.x0_given = 0
        st = (SolverStats * nrhs)()
        rc = _lib.load().wc_fgmres_dr_solve(self._ctx, _ptr(x), _ptr(b), nrhs, ctypes.byref(p), int(k), st,
                                            _stream(stream))
        stats = [s.as_dict() for s in st]
        if check:
            _lib.check(rc)
        return x, stats

    def link_grad(self, Y, X, coef=1.0, stream=None):
        """G with d(sum Re<Y, D X>) = Re sum tr(G^dag dU), times coef (torch gradient convention)."""
        nrhs = self._spinor(X, "X")
        self._spinor(Y, "Y", like=X)
        torch = _torch()
        G = torch.empty_like(self._U)
        _lib.check(_lib.load().wc_link_grad(self._ctx, _ptr(G), _ptr(Y), _ptr(X), nrhs, float(coef),
                                            _stream(stream)))
        return G

    def force(self, phi, params: SolverParams | None = None, stream=None, **kw):
        """Pseudofermion force of S = phi^dag (D^dag D)^-1 phi for one pseudofermion field
        phi [L0..L3][4][3]; returns (F, Y, X, stats)."""
        if self._spinor(phi, "phi") != 1 or phi.dim() != 6:
            raise WCError(-1, f"phi must be one field [L0..L3][4][3], got {tuple(phi.shape)}")
        torch = _torch()
        p = _params(params, kw)
        F = torch.empty_like(self._U)
        Y = self.new_spinor()
        X = self.new_spinor()
        st = (SolverStats * 2)()
        _lib.check(_lib.load().wc_force(self._ctx, _ptr(F), _ptr(phi), ctypes.byref(p), st, _ptr(Y), _ptr(X),
                                        _stream(stream)))
        return F, Y, X, [s.as_dict() for s in st]

    def autotune(self, nrhs, prec="f32", stream=None):
        """Tune the rhs tiles for solves of nrhs rhs whose preconditioner runs in prec.
        Returns (D tile in prec, FP64 D tile, plain block-solver tile, even/odd tile)."""
        out = (ctypes.c_int * 4)()
        _lib.check(_lib.load().wc_autotune(self._ctx, int(nrhs), PREC[prec], out, _stream(stream)))
        return tuple(int(v) for v in out)

    def set_option(self, name, value):
        """Kernel choice of this context: "sap_cache" or "dirac_stage", -1 (automatic), 0 or 1."""
        _lib.check(_lib.load().wc_set_option(self._ctx, _lib.OPTIONS[name], int(value)))

    def set_tiles(self, prec, nr_dirac=0, nr_sap=0, nr_sap_eo=0):
        """Right-hand sides handled together in precision prec (0: the library's choice)."""
        _lib.check(_lib.load().wc_set_tiles(self._ctx, PREC[prec], int(nr_dirac), int(nr_sap), int(nr_sap_eo)))

    def action(self, phi, params: SolverParams | None = None, stream=None, **kw):
        """Pseudofermion action S = phi^dag (D^dag D)^-1 phi = |Y|^2 for one field phi;
        returns (S, Y, X, stats) with Y = D^-dag phi and X = D^-1 Y."""
        if self._spinor(phi, "phi") != 1 or phi.dim() != 6:
            raise WCError(-1, f"phi must be one field [L0..L3][4][3], got {tuple(phi.shape)}")
        p = _params(params, kw)
        Y = self.new_spinor()
        X = self.new_spinor()
        S = ctypes.c_double()
        st = (SolverStats * 2)()
        _lib.check(_lib.load().wc_pseudofermion_action(self._ctx, _ptr(phi), ctypes.byref(p), ctypes.byref(S),
                                                       _ptr(Y), _ptr(X), st, _stream(stream)))
        return S.value, Y, X, [s.as_dict() for s in st]

    def scale(self, x, coef, out=None, stream=None):
        """out = coef * x for spinor fields of this lattice."""
        nrhs = self._spinor(x, "x")
        if out is None:
            out = self.new_spinor(None if x.dim() == 6 else nrhs)
        else:
            self._spinor(out, "out", like=x)
        _lib.check(_lib.load().wc_spinor_scale(self._ctx, _ptr(out), _ptr(x), nrhs, float(coef), _stream(stream)))
        return out

    def autotune_block(self, params: SolverParams | None = None, stream=None, **kw):
        p = _params(params, kw)
        out = (ctypes.c_int * 4)()
        _lib.check(_lib.load().wc_autotune_block(self._ctx, ctypes.byref(p), out, _stream(stream)))
        self.block = tuple(int(v) for v in out)
        return self.block

    def set_block(self, block, stream=None):
        blk = (ctypes.c_int * 4)(*block)
        _lib.check(_lib.load().wc_set_block(self._ctx, blk, _stream(stream)))
        self.block = tuple(int(b) for b in block)

    def bench_dirac(self, prec="f64", nrhs=1, region="full", iters=50, stream=None):
        ms = ctypes.c_double()
        _lib.check(_lib.load().wc_bench_dirac(self._ctx, PREC[prec], int(nrhs), REGION[region], int(iters),
                                              ctypes.byref(ms), _stream(stream)))
        return ms.value

    def bench_sap(self, prec="f32", nrhs=1, nmr=4, iters=20, eo=False, stream=None):
        ms = ctypes.c_double()
        _lib.check(_lib.load().wc_bench_sap(self._ctx, PREC[prec], int(nrhs), int(nmr), int(bool(eo)), int(iters),
                                            ctypes.byref(ms), _stream(stream)))
        return ms.value


def solve_batch(lattices, bs, params: SolverParams | None = None, stream=None, check=True, k=None, **kw):
    """Solve several lattices (possibly of different sizes) in one batched solve: FGCR, or
    FGMRES-DR keeping k harmonic Ritz vectors when k is given.

    bs[i] is a complex128 [nrhs_i][dims_i][4][3] tensor.  Returns (xs, stats)."""
    lib = _lib.load()
    n = len(lattices)
    if len(bs) != n:
        raise WCError(-1, f"{len(bs)} source tensors for {n} lattices")
    p = _params(params, kw)
    p.x0_given = 0
    xs, nr = [], []
    for lat, b in zip(lattices, bs):
        nr.append(lat._spinor(b, "b"))
        xs.append(lat.new_spinor(None if b.dim() == 6 else nr[-1]))
    ctxs = (ctypes.c_void_p * n)(*[lat._ctx.value for lat in lattices])
    xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
    nrhs = (ctypes.c_int * n)(*nr)
    st = (SolverStats * sum(nr))()
    if k is None:
        rc = lib.wc_fgcr_solve_batch(ctxs, n, xp, bp, nrhs, ctypes.byref(p), st, _stream(stream))
    else:
        rc = lib.wc_fgmres_dr_solve_batch(ctxs, n, xp, bp, nrhs, ctypes.byref(p), int(k), st, _stream(stream))
    if check:
        _lib.check(rc)
    return xs, [s.as_dict() for s in st]
