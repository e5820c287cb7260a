"""FP64 CPU oracle for the spectral-element Poisson operator and Jacobi-PCG.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
bench's CPU-baseline leg may import this package.  The GPU library shares no
code with it and never calls it.

It is a plain, slow, readable NumPy implementation in float64 of what the
Nekbone workload of the paper computes (Sec. VIII-A: Jacobi-preconditioned CG
for a 3-D Poisson problem on a box of E hexahedra, each with (N+1)^3 nodes of
an order-N tensor basis; the ``ax`` Poisson-operator kernel and the ``gs``
gather-scatter of Sec. V-B / Fig. kernel_transform; the CG dot-product tree
reductions and streaming kernels of Sec. VIII-B).  The paper prints none of
the formulas; they are the standard nodal spectral-element method on
Gauss-Lobatto-Legendre points, and every function says which step it takes.

Modules
-------
gll       GLL nodes/weights and the 1-D derivative matrix.
mesh      box-mesh coordinates, global node ids, Dirichlet mask.
operator  geometric factors, element operator A_L, dssum, Jacobi diagonal.
pcg       Jacobi-preconditioned CG with multiplicity-weighted dots.
dots      exactly rounded dot products (error-free transforms + fsum).
brute     dense element matrices from a Legendre-Vandermonde basis.
mixed     low-precision operator emulation and inner-outer refinement.
gs        generic gather-scatter in compressed-row form (any id map).

Parity status: every function here is pinned by a test of the CPU suite
against a closed form, a library routine at higher precision, a dense brute
force or an invariant, except the iterates of the low-precision inner solver,
which are "parity unpinned" (only their FP64 outer result is pinned).
"""

from . import gll, mesh, operator, pcg, dots, brute, mixed, gs  # noqa: F401
