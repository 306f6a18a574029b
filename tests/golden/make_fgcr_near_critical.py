"""Write fgcr_near_critical_8x8x8x8.txt: the oracle's FP64 SAP-FGCR close to the critical mass.

On the 8^4 lattice (gauge recipe eps = 0.3, seed 1234; Gaussian source, seed 5678;
m0 = -0.17, c_sw = 1, periodic) the smallest real part of the spectrum sits about 0.01
above zero, the near-critical regime of Sec. 4 (Fig. 1), where restarted FGCR needs many
cycles and Gram-Schmidt cancels most of each new direction.  The oracle's FGCR (modified
Gram-Schmidt, restart 16; SAP with 4^4 blocks, 4 block-solver steps, 5 cycles; tol 1e-10)
runs once with the plain MR block solver and once with the even/odd one.  Each row:
eo iterations restarts, then the relative true residual after each restart.  Calls only
the oracle.

    PYTHONPATH=. python tests/golden/make_fgcr_near_critical.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import synth  # noqa: E402
from oracle import dirac, solvers  # noqa: E402

DIMS, BLOCK = (8, 8, 8, 8), (4, 4, 4, 4)
M0, CSW = -0.17, 1.0


def main():
    U = synth.gauge_field(DIMS)
    A = dirac.clover_matrix(U, M0, CSW)
    b = synth.gaussian_spinor(DIMS)
    rows = ["# eo iters restarts | relative true residual after each restart; SAP-FGCR(16) of the oracle, "
            "8^4, m0=-0.17, c_sw=1, 4^4 blocks, nmr=4, ncy=5, tol=1e-10; written by make_fgcr_near_critical.py"]
    for eo in (0, 1):
        r = solvers.sap_fgcr(U, A, b, BLOCK, nmr=4, ncy=5, nkv=16, tol=1e-10, eo=bool(eo))
        assert r.converged
        rows.append(f"{eo} {r.iters} {r.restarts} | " + " ".join(f"{h:.17e}" for h in r.history[1:]))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fgcr_near_critical_8x8x8x8.txt")
    open(out, "w").write("\n".join(rows) + "\n")


if __name__ == "__main__":
    main()
