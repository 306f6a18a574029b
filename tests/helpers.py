"""Shared helpers of the GPU parity tests: seeded inputs on the device, oracle references."""
import functools

import numpy as np

import synth
from oracle import dirac


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def to_dev(a):
    torch, dev = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_np(t):
    return t.detach().cpu().numpy()


@functools.lru_cache(maxsize=8)
def gauge(dims, eps=0.3, seed=synth.GAUGE_SEED):
    return synth.gauge_field(dims, eps=eps, seed=seed)


@functools.lru_cache(maxsize=8)
def clover(dims, m0, csw, eps=0.3, seed=synth.GAUGE_SEED):
    return dirac.clover_matrix(gauge(dims, eps, seed), m0, csw)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def lattice(dims, block, m0=-0.1, csw=1.0, bc_t=1, seed=synth.GAUGE_SEED):
    import paper_1109_4279_amd as wc
    return wc.Lattice(to_dev(gauge(dims, 0.3, seed)), block=block, m0=m0, csw=csw, bc_t=bc_t)


# ----------------------------------------------------------------- the oracle's D on time slabs

HALO = 2  # the clover term at x reads links one step away in every direction, D one more


def _slab_task(args):
    """Oracle D x on time layers [t0, t0 + T) of a periodic lattice: the slab with HALO layers
    on each side is taken as its own periodic lattice; its wrap corrupts only the halo."""
    U_slab, xs, m0, csw = args
    A = dirac.clover_matrix(U_slab, m0, csw)
    return [dirac.apply_D(U_slab, A, x)[HALO:-HALO] for x in xs]


def oracle_D_slabs(U, xs, m0, csw, starts=None, T=4, workers=8):
    """The oracle's FP64 D applied to each field of xs (lists of [L0..L3][4][3] arrays,
    periodic in time) on the time layers [t0, t0 + T) for t0 in starts (every slab by
    default), as a dict t0 -> list of arrays [T][L1][L2][L3][4][3].  Slabs run in a pool
    of worker processes that touch no GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    L0 = U.shape[1]
    if starts is None:
        starts = list(range(0, L0, T))
    tasks = []
    for t0 in starts:
        idx = np.arange(t0 - HALO, t0 + T + HALO) % L0
        tasks.append((np.ascontiguousarray(U[:, idx]), [np.ascontiguousarray(x[idx]) for x in xs], m0, csw))
    if workers <= 1 or len(tasks) == 1:
        return {t0: _slab_task(t) for t0, t in zip(starts, tasks)}
    with cf.ProcessPoolExecutor(min(workers, len(tasks)), mp_context=mp.get_context("spawn")) as ex:
        return dict(zip(starts, ex.map(_slab_task, tasks)))


def oracle_true_res(U, m0, csw, xs, bs, T=4, workers=8):
    """|b - D x| / |b| with the oracle's D for each pair (x, b), from slabs covering the lattice."""
    L0 = U.shape[1]
    got = oracle_D_slabs(U, xs, m0, csw, list(range(0, L0, T)), T, workers)
    out = []
    for i, b in enumerate(bs):
        r2 = 0.0
        for t0, ds in got.items():
            r = b[t0:t0 + T] - ds[i]
            r2 += float(np.vdot(r, r).real)
        out.append(np.sqrt(r2) / np.linalg.norm(b.ravel()))
    return out
