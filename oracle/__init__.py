"""CPU FP64 oracle for the ghost-FEM multigrid solver (test infrastructure).

This package is the plain, slow reference implementation that the HIP path is
checked against.  It is test infrastructure only: the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it; the product path never
imports, calls or links it, and it shares no code with the HIP kernels.

Layout (all numpy / scipy, float64):

* ``geometry``   snapping, cell classification, cut fractions, cut polygons and
                 interface segments, the stabilisation constant C(K)
                 (section 2; section 5.2 "Global and local stabilization
                 parameters", eqs. c_triangle / c_pentagon and the
                 quadrilateral formula)
* ``quadrature`` exact integration of Q1 basis products on polygons/segments
* ``assembly``   element matrices and global sparse A, M, G, the Neumann
                 load GN of mixed boundaries (eqs. disc_bil_form / disc_rhs),
                 the global generalised eigenproblem of section 5.2
* ``multigrid``  bilinear prolongation, Galerkin hierarchy (eq. galerkin),
                 four-colour and lexicographic Gauss-Seidel, extra smoothing on
                 cut cells, two-grid scheme (Algorithm 1), V- and W-cycles,
                 convergence factors (section 3)
* ``adjoint``    misfit, transposed V-cycle, gradients w.r.t. f, g and g_N

Readings where the paper is silent are stated at the function that implements
each of them.
"""
from . import geometry, quadrature, assembly, multigrid, adjoint  # noqa: F401
