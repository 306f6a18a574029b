"""wc_apply_D_noalloc through the C interface: the same output as wc_apply_D, bit for bit,
on two calls in a row (the second with a smaller input), in every storage precision, for
the full and the block operator and for D^dag; requests beyond its scratch are rejected."""
import ctypes

import numpy as np
import pytest

import synth
from tests.helpers import lattice, to_dev, to_np

pytestmark = pytest.mark.gpu


def _c_apply(fn, lat, x, prec, region, dagger):
    from paper_1109_4279_amd import PREC, REGION, _lib
    nrhs = 1 if x.dim() == 6 else x.shape[0]
    out = lat.new_spinor(None if x.dim() == 6 else nrhs)
    import torch
    rc = fn(lat._ctx, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs, PREC[prec],
            REGION[region], int(dagger), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, _lib.load().wc_last_error()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_noalloc_equals_apply_D(prec):
    from paper_1109_4279_amd import _lib
    lib = _lib.load()
    for dims, block in (((8, 8, 8, 8), (4, 4, 4, 4)), ((8, 6, 6, 6), (4, 3, 3, 3))):
        lat = lattice(dims, block)
        big = to_dev(synth.gaussian_spinor(dims, nrhs=3, seed=91))
        small = to_dev(synth.gaussian_spinor(dims, seed=92))
        for region, dagger in (("full", 0), ("blocks", 0), ("full", 1)):
            for x in (big, small):  # two calls in a row, the second smaller
                want = to_np(_c_apply(lib.wc_apply_D, lat, x, prec, region, dagger))
                got = to_np(_c_apply(lib.wc_apply_D_noalloc, lat, x, prec, region, dagger))
                assert np.array_equal(got, want), (dims, region, dagger, x.dim())


def test_noalloc_errors():
    import torch

    from paper_1109_4279_amd import PREC, _lib
    lib = _lib.load()
    dims = (32, 16, 16, 16)
    lat = lattice(dims, (4, 4, 4, 4))
    x = lat.new_spinor(3)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(x.data_ptr())
    # 3 FP64 rhs of 16^3 x 32 need 144 MiB of scratch, above the 128 MiB it holds
    assert lib.wc_apply_D_noalloc(lat._ctx, p, p, 3, PREC["f64"], 0, 0, s) == -1
    assert b"MiB" in lib.wc_last_error()
    # the FP32 operator has not been built on this context yet
    assert lib.wc_apply_D_noalloc(lat._ctx, p, p, 1, PREC["f32"], 0, 0, s) == -7
    assert lib.wc_apply_D_noalloc(None, p, p, 1, 0, 0, 0, s) == -1
