"""Plain FP64 CPU oracle of the agglomeration multigrid for Compact DG (CDG).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the GPU library never
does, and this package never imports the library.

It follows Pan & Persson, "Agglomeration-based geometric multigrid solvers
for compact discontinuous Galerkin discretizations on unstructured meshes":

* ``refelem``     reference simplex, quadrature and the nodal P_p basis (Sec. 2.2)
* ``mesh``        facet table of a simplex mesh
* ``switch``      CDG switch functions: natural and consistent (Sec. 2.2, Sec. 4.2)
* ``cdg``         CDG primal operator A, flux form M, G, C (Sec. 2.2-2.3)
* ``agglomerate`` greedy agglomeration, Alg. 1 and Alg. 2 (Sec. 3.1-3.2)
* ``multigrid``   agglomerate bases, transfers, flux/primal coarsening, the
                  V-cycle with damped block Jacobi (Sec. 3.3-3.5, Sec. 4.1, Alg. 3);
                  the hp front end, p-multigrid down to p = 1 by nodal
                  embeddings before the agglomeration levels (Sec. 4, hp
                  paragraph)
* ``krylov``      PCG, flexible CG (FCG(1), Notay 2000) and right-preconditioned
                  GMRES(m) (Sec. 4) outer solvers
* ``adjoint``     adjoint gradients dL/dkappa and dL/df of the solve

Every function computes in float64 with plain NumPy / SciPy primitives and
no blocking or fusion.  Pins that fix each part independently of this code
live in ``tests/test_oracle_*.py``.  The agglomeration's element->aggregate
maps beyond the structured-grid case are "parity unpinned" by the paper
(it prints no maps); see the module docstring of ``agglomerate``.
"""
