"""CPU FP64 oracle for the H-matrix BEM hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy implementation of what
the HIP library computes, written from the paper (Harbrecht & Zaspel,
"A scalable H-matrix approach for the solution of boundary integral
equations on multi-GPU clusters", arXiv 1806.11558) and the collocation
discretisation the library implements.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library and its
Python binding never do, and it shares no code with them.

Modules
  quadrature  Radon's degree-5 seven-point triangle rule.
  bem         Laplace single-layer collocation operator (Sec. 2.1, Example 1):
              centroids, areas, quadrature nodes, analytic self-term, matrix
              entries, dense matrix, exact rows/columns, direct products,
              single-layer potential at interior points.
  cluster     Morton codes and sort (Sec. 3.1 "Spatial data structure"),
              cardinality-based cluster tree (Sec. 2.3, (C1)-(C4)), bounding
              boxes and admissibility (Sec. 2.3, eq. admissibilityCondition),
              block cluster tree (Sec. 2.3, Algorithm 1).
  aca         Adaptive cross approximation with partial pivoting (Sec. 2.3).
  galerkin    The paper's own Galerkin discretisation (Sec. 2.2, eq.
              linearSystem) with piecewise constants: 7 x 7 rule for pairs
              that share no vertex, outer Gauss rule with the inner integral
              in closed form (the Duffy / polar split, Sec. 4.1) for
              touching pairs; right-hand sides; the potential for the
              interior error eps(h) of Sec. 4.3.
  sphere      Closed forms on the unit sphere used as pins.

Parity unpinned: the exact discretisation-error values at each refinement
level (the paper prints none for this discretisation); they are checked as
convergence trends only.
"""
