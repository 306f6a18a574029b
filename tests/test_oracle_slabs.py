"""The oracle's D on time slabs with halos (the route the 32^3 x 64 GPU parity tests take)
equals the oracle's D on the whole lattice."""
import numpy as np

import synth
from oracle import dirac
from tests.helpers import oracle_D_slabs, oracle_true_res


def test_slabs_equal_whole_lattice():
    dims, m0, csw = (8, 4, 4, 4), -0.1, 1.0
    U = synth.gauge_field(dims)
    x = synth.gaussian_spinor(dims, seed=3)
    y = synth.gaussian_spinor(dims, seed=4)
    A = dirac.clover_matrix(U, m0, csw)
    want = [dirac.apply_D(U, A, x), dirac.apply_D(U, A, y)]
    got = oracle_D_slabs(U, [x, y], m0, csw, T=2, workers=1)
    assert sorted(got) == [0, 2, 4, 6]
    for t0, ds in got.items():
        for w, d in zip(want, ds):
            assert np.abs(d - w[t0:t0 + 2]).max() < 1e-14 * np.abs(w).max()
    # the slab residual of the exact answer's source is the residual of the whole lattice
    b = want[0] + 1e-3 * y
    res = oracle_true_res(U, m0, csw, [x], [b], T=4, workers=2)[0]
    assert abs(res - 1e-3 * np.linalg.norm(y) / np.linalg.norm(b)) < 1e-12
