"""Euclidean Dirac matrices in a chiral basis (oracle; test infrastructure only).

The paper (abstract, Sec. 4) names the Wilson-Dirac operator with clover term but
never writes a gamma basis.  The clover term is stored as two 6x6 Hermitian
chiral blocks per site, which requires gamma_5 to be diagonal; the reading used
throughout is

    gamma_0 = [[0, -1], [-1, 0]],   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],

in 2x2 spin blocks, so that gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1, 1, -1, -1).
Index 0 is the time direction.
"""
from __future__ import annotations

import numpy as np

PAULI = np.array(
    [
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)
I2 = np.eye(2, dtype=np.complex128)
Z2 = np.zeros((2, 2), dtype=np.complex128)


def _blocks(a, b, c, d):
    return np.block([[a, b], [c, d]])


def gammas() -> np.ndarray:
    """gamma_mu for mu = 0..3, shape (4, 4, 4)."""
    g = np.empty((4, 4, 4), dtype=np.complex128)
    g[0] = _blocks(Z2, -I2, -I2, Z2)
    for k in range(3):
        g[k + 1] = _blocks(Z2, -1j * PAULI[k], 1j * PAULI[k], Z2)
    return g


GAMMA = gammas()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]."""
    g = GAMMA
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
