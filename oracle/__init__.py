"""CPU FP64 oracle for the graph-based S_N transport sweep on curved meshes.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never does, and
the two share no code (only the seeded input generators in ``workloads``).

Modules, each following the paper (Haut et al., "An Efficient Sweep-based
Solver for the S_N Equations on High-Order Meshes"):

* ``quadrature`` -- level-symmetric S_N directions and weights (section 2,
  quadrature assumptions under eq. linearSnTransport).
* ``basis``      -- 1D Gauss rules and Lagrange bases (section 2, eqs.
  elementTransformation and localBasis).
* ``geometry``   -- element maps, Jacobians, mass and gradient moments
  (eqs. Jacobian, localMtMatrix, localGMatrix).
* ``faces``      -- face normals and the upwind face integrals with their
  sign changes on curved faces (eqs. localFDiagonalMatrix,
  localFOffDiagonalMatrix and the discussion of non-smooth integrands).
* ``graph``      -- per-direction dependency graph, edge weights, Tarjan
  SCCs, minimum feedback arc sets, levels (section 3, eq. graphWeight).
* ``sweep``      -- lagged transport sweep and source iteration
  (eqs. sourceIteration, fSplitting, laggedSourceIteration).
* ``dense``      -- brute-force global solve of eq. matrixFormLinearTransport.
* ``mixed``      -- FP32 local solve with one FP64 refinement step.

Readings where the paper is silent or its print is garbled are stated in each
function's docstring.
"""
from .quadrature import level_symmetric
from .discretization import Discretization
from .graph import direction_graph, GraphResult
from .sweep import sweep, source_iteration

__all__ = ["level_symmetric", "Discretization", "direction_graph",
           "GraphResult", "sweep", "source_iteration"]
