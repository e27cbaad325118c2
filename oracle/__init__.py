"""Plain FP64 CPU oracle for the Kohn-Sham direct minimisation on the Stiefel manifold.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
the benchmark's CPU-baseline leg may import or run anything in this folder.
The product path (the HIP library and its Python binding) never calls it.

What it implements (Zhang, Zhu, Wen, Zhou, "Gradient type optimization methods
for electronic structure calculations"):

* ``fd``      uniform-grid discretisation: -Laplacian by the 7-point stencil with
              zero Dirichlet boundary, erf-smoothed nuclear potential, nuclear
              repulsion (Section 2.1 eq. (EKS), Section 2.3).
* ``ks``      density rho(X) = diag(XX^T) (scaled), Hartree potential by
              warm-started conjugate gradients, Slater exchange, the discrete
              energy (Section 2.3) and its partial derivative E_X = H(X)X
              (eq. (partial deriv)).
* ``stiefel`` manifold gradient (eq. (def-nablaE)), the QR retraction via
              Cholesky QR (eq. (QR), Alg. 2), the Cayley retraction in
              Sherman-Morrison-Woodbury form (eqs. (WY1), (WY3)).
* ``optm``    Alg. 3: Barzilai-Borwein step (eq. (bb-1)), nonmonotone Armijo
              search (eq. (NMLS-Armijo)), stopping rules of Section 4.1.
* ``fe``      trilinear (Q1) finite elements on a uniform hexahedral mesh with
              the consistent mass matrix B and the B-orthonormality constraint
              (Section 2.3 finite-element form, Section 3 eq. (OFDFT-y)).
* ``precision`` bfloat16 rounding and the Gram blocks of rounded operands (the
              tall-skinny products of Section 3 in a reduced-precision mode).

Everything is float64 and written for clarity, not speed: no blocking, fusion or
reordering beyond what the definitions state.
"""
