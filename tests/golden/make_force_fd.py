"""Write force_fd_4x4x4x4.txt: central finite differences of the pseudofermion action.

S(U) = phi^dag (D^dag D)^-1 phi on the 4^4 lattice (gauge recipe eps = 0.3, seed 1234;
phi Gaussian, seed 4321; m0 = -0.1, c_sw = 1, periodic), evaluated by the oracle's dense
LU, at U_mu(x) -> exp(+-h T^a) U_mu(x) with h = 1e-6, for 8 sampled links x all 8
generators.  Each row: mu x0 x1 x2 x3 a  (S+ - S-)/(2h).  Calls only the oracle.

    PYTHONPATH=. python tests/golden/make_force_fd.py
"""
import os
import sys

import numpy as np
import scipy.linalg as sla

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import synth  # noqa: E402
from oracle import dense, force  # noqa: E402

DIMS = (4, 4, 4, 4)
M0, CSW, H = -0.1, 1.0, 1e-6


def main():
    U = synth.gauge_field(DIMS)
    phi = synth.gaussian_spinor(DIMS, seed=synth.FORCE_PHI_SEED)
    T = force.su3_generators()
    rng = np.random.default_rng(synth.FORCE_PHI_SEED)
    rows = []
    for _ in range(8):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(d)) for d in DIMS)
        idx = (mu,) + site
        for a in range(8):
            s = []
            for sign in (1, -1):
                Up = U.copy()
                Up[idx] = sla.expm(sign * H * T[a]) @ U[idx]
                s.append(dense.action(Up, M0, CSW, phi))
            rows.append(list(idx) + [a, (s[0] - s[1]) / (2 * H)])
            print(rows[-1], flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "force_fd_4x4x4x4.txt")
    np.savetxt(out, np.array(rows), fmt=["%d"] * 6 + ["%.17e"],
               header="mu x0 x1 x2 x3 a dS/deps_a (central difference, h=1e-6); "
                      "written by make_force_fd.py from the oracle's dense action")


if __name__ == "__main__":
    main()
