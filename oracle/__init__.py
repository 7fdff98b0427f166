"""Reference oracle for weighted-Gaussian row-wise assembly (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, independent restatement of what the method of
Barton, Puzyrev, Deng and Calo, "Efficient mass and stiffness matrix assembly via
weighted Gaussian quadrature rules for B-splines" (arXiv 1710.01048) computes:

* ``oracle.bspline`` -- Cox-de Boor B-spline values and derivatives on open
  uniform knot vectors (Sec. 2.2, eq:Gmap3).
* ``oracle.rules``   -- the weighted Gaussian rules, solved from the exactness
  systems eq:GaussQuadSys (mass, Sec. 3.1) and eq:GaussQuadSysStiff (stiffness,
  Sec. 3.2) in high precision, plus the boundary-row rules the paper leaves open
  (Remark at the end of Sec. 3.2).
* ``oracle.assemble`` -- FP64 direct (not sum-factorized) row-wise sums for the
  mass matrix (eq:Mass), the stiffness matrix with diagonal coefficient
  (eq:Stiffness) and the adjoint of both, in plain C with OpenMP over rows.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in here.  The product library never
does, and this package imports nothing from the product package.
"""
