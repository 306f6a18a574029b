"""Host-side dense algebra of the library's FGMRES-DR restarts against the oracle (no GPU):
the C entry point wc_harmonic_ritz runs on the CPU."""
import ctypes
import os

import numpy as np
import pytest

from oracle import solvers


def _lib():
    from paper_1109_4279_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwc.so not built")
    return _lib.load()


def _arnoldi_hbar(n, m, seed, small=()):
    """Hbar of m Arnoldi steps (modified Gram-Schmidt) on a random non-normal matrix."""
    rng = np.random.default_rng(seed)
    lam = 1.0 + rng.random(n) + 0.3j * (rng.random(n) - 0.5)
    lam[: len(small)] = small
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = Q @ np.diag(lam) @ Q.conj().T + 0.2 * np.triu(rng.standard_normal((n, n)), 1) / n
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V = [v / np.linalg.norm(v)]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    for j in range(m):
        w = A @ V[j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
    return H


@pytest.mark.parametrize("m,seed", [(1, 1), (4, 2), (8, 3), (16, 4), (32, 5)])
def test_harmonic_ritz_matches_oracle(m, seed):
    lib = _lib()
    H = _arnoldi_hbar(80, m, seed, small=(0.01, 0.02 + 0.01j, -0.015j))
    # a deflated restart leaves a dense leading block: mix the first columns
    if m >= 4:
        rng = np.random.default_rng(seed + 100)
        Qk, _ = np.linalg.qr(rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
        H[:4, :3] = H[:4, :3] @ Qk
    Hf = np.asfortranarray(H)
    theta = np.zeros(m, dtype=np.complex128)
    G = np.zeros((m, m), dtype=np.complex128, order="F")
    rc = lib.wc_harmonic_ritz(m, Hf.ctypes.data_as(ctypes.c_void_p), theta.ctypes.data_as(ctypes.c_void_p),
                              G.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    tw, Gw = solvers.harmonic_ritz(H)
    assert np.allclose(np.abs(theta), np.abs(tw), rtol=1e-10, atol=1e-13)
    assert np.abs(theta - tw).max() < 1e-9 * np.abs(tw).max()
    for i in range(m):
        # unit eigenvectors agree up to a phase (eigenvalues are distinct here)
        assert abs(abs(np.vdot(G[:, i], Gw[:, i])) - 1.0) < 1e-8
        assert abs(np.linalg.norm(G[:, i]) - 1.0) < 1e-12


def test_harmonic_ritz_rejects_bad_input():
    lib = _lib()
    H = np.zeros((3, 2), dtype=np.complex128, order="F")
    out = np.zeros(4, dtype=np.complex128)
    assert lib.wc_harmonic_ritz(0, H.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                                out.ctypes.data_as(ctypes.c_void_p)) == -1
    # singular H: no harmonic Ritz pairs
    assert lib.wc_harmonic_ritz(2, H.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                                out.ctypes.data_as(ctypes.c_void_p)) == -6
