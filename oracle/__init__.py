"""Plain FP64 CPU oracle for n-gluon tree amplitudes (TEST INFRASTRUCTURE).

This package is test infrastructure.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import or run
it.  The HIP library never calls it and shares no code with it: the two are
separate implementations of the same definitions, and the oracle is pinned to
closed forms and identities by the CPU tests.

Contents (each module cites the passage of the paper it follows):
  dual          first-order dual numbers (forward-mode derivatives)
  lorentz       Minkowski products, metric (+,-,-,-)
  polarization  helicity vectors and the light-cone projector (Section 2.1)
  cobg          colour-ordered Berends-Giele currents and partial amplitudes
                (Section 2.3), explicit four-gluon vertex and tensor form
  color         colour coefficients of the adjoint decomposition (Section 2.2)
  me2           colour- and helicity-summed |M|^2 (Section 2.2)
  cdbg          colour-dressed recursion in the colour-flow basis (Section 2.3)
                and the brute-force colour-flow sum (Section 2.2)
  cdmc          the dressed recursion with continuous colour vectors and real
                polarizations (Section 2.1)
  grad          d|M|^2/dp from forward-mode dual numbers
Every function works in float64 / complex128 numpy arrays vectorised over
events (the last axis); nothing is blocked, fused or reordered beyond the
definitions.
"""
