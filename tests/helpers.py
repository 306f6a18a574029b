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
