"""FP64 CPU oracle for the explicit upwind DG elastic-wave right-hand side.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP library and
its Python binding never import it, and this package imports nothing from
them: the two share no kernels, helpers, tables or constants.

The oracle is written for clarity, not speed: a modal Galerkin method with the
orthonormal Dubiner (Proriol-Koornwinder) basis of P_N, built from Jacobi
polynomials in collapsed coordinates (values from scipy.special.eval_jacobi),
every integral evaluated by quadrature (Gauss-Jacobi nodes from
scipy.special.roots_jacobi), faces matched by physical coordinates.  The GPU path instead uses a nodal basis, derivative/lift
matrices and topological face permutations.  Both discretise the same
semi-discrete operator, which does not depend on the basis:

* the first-order system  sum_k d_k(A_k u) + C u = f  (Sec. 2, eq. LPDE) with
  the elastic velocity-strain instance (C = 0);
* the upwind HDG flux  F^.n = F(u).n + |A|(u - u^)  (Sec. 2, eq.
  RiemannFluxBoth) with the trace u^ eliminated through the single-valued
  trace condition (Sec. 2, eq. HDGeqn; Sec. 3, eq. iHDGtrace), generalised
  to different impedances on the two sides of a face;
* the element-by-element explicit update of Sec. 4.3 with forward Euler
  replaced by a five-stage low-storage Runge-Kutta scheme;
* the implicit (theta-scheme) step of the same operator solved by iHDG-II
  (Sec. 3, Algorithm 1; ihdg.py);
* steady transport by upwind HDG on structured squares and cubes solved by
  iHDG-II (Sec. 4.1, Sec. 6.1; transport.py).

Parity status: every function is pinned by tests under tests/ (exactness,
closed-form energy rate, conservation, plane-wave convergence, symmetry,
Runge-Kutta order conditions, receiver sampling time against an exact
wave; for iHDG-II a Krylov solve of the global implicit system, the theta
scheme's discrete energy identities and its order in time; for transport
the paper's printed iteration counts, the marching of Theorem 1, a direct
solve, exactness on Q_p and the order of accuracy).  Absolute
solution values of the large heterogeneous workloads are not printed in the
paper and are pinned only through those properties.
"""

