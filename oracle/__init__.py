"""FP64 CPU oracle for the contour-integral sign function and overlap operator.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or
executes anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library: no
kernels, headers, tables or helpers.  Its only common dependency is the seeded
input generator (``seeded_inputs``), which holds none of the method's
arithmetic.

What it computes (plain numpy/scipy, complex128 throughout):

* ``wilson.hermitian_wilson`` -- H_W = gamma5 D_W(-m0) as a sparse CSR matrix
  written out from the hopping formula (eq. (1) and the definition of H_W
  below it), with the normalisation D_W = 1 - kappa * hop,
  kappa = 1/(2(4 - m0)).
* ``contour.nodes`` -- the N_q-point trapezoidal nodes z_j and weights
  rho w_j / N_q on the ellipses Gamma_+ and Gamma_- (eq. (7)); the weights of
  Gamma_- carry the minus sign of eq. (3).
* ``sign.sign_by_solves`` -- sum_j c_j y_j with every shifted system
  (z_j I - H_W) y_j = b (eq. (6)) solved on its own by a dense or sparse LU
  solve, or by restarted GMRES(100) accepted only when its true residual is
  below 10 rtol (eqs. (5)-(7)).
* ``sign.sign_by_eigh`` -- the same rational filter, and the exact sign, from a
  dense eigendecomposition (eq. (2)); small lattices only.
* ``sign.overlap`` -- D_ov(m_q) b = (1+m_q)/2 b + (1-m_q)/2 gamma5 s (eq. (1)).
* ``freefield`` -- unit-link closed forms in momentum space (any size).
* ``force`` -- the derivative of phi^dag D_ov^dag D_ov phi with respect to the
  links, by the adjoint-solve formula and by dense finite differences.

Readings where the paper is silent (normalisation of D_W, gamma basis, sign of
the projectors, boundary conditions, what N_q counts) are stated in the
function docstrings.  Every function here is pinned by the ``-m "not gpu"``
tests against closed forms, invariants or brute force.
"""
