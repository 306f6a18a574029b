"""Plain FP64 CPU oracle for the Wilson-clover SAP-FGCR hot path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
anything in this package.  The library never calls it, shares no code with it,
and fails loudly if its own compiled extension is missing.

Contents (every function cites the passage of arXiv:1109.4279 it follows):

* ``gamma``   - the chiral Euclidean gamma basis and sigma_{mu nu}.
* ``dirac``   - clover field strength, the clover matrix, D_w on the full lattice
                and on Dirichlet blocks (Sec. 4, the Wilson-Dirac operator with
                clover term of the abstract).
* ``solvers`` - block MR, the Schwarz alternating procedure and restarted FGCR
                (Sec. 4).
* ``force``   - the gauge-link derivative of S = phi^dag (D^dag D)^-1 phi
                (the HMC force that motivates the solves, Sec. 1).
* ``dense``   - dense-matrix assembly for brute-force checks on tiny lattices.

Everything is complex128 numpy with the array conventions of ``synth``.
"""
