"""FP64 complex CPU oracle for four-component LR-CCSD polarizabilities.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls anything in this package.  Only
the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the bench
use it.  It shares no code with the HIP path: it takes plain arrays from the
seeded generator and computes everything itself, slowly and densely, in
complex128 with PyTorch CPU ops (einsum, autograd) and numpy.

Modules
-------
integrals   antisymmetrized spinor integrals from density-fitting factors
ccsd        CCSD residual Omega(t), energy E(t), packed amplitude layout
derivs      Jacobian-vector products (contour rule, forward mode) and
            transposed products (reverse mode)
response    T, Lambda, X(omega), Y(omega) solves and the polarizability
detspace    brute-force determinant-space CC and FCI sum-over-states (pins)
fnspp       perturbation-sensitive natural spinor truncation (FNS++)

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (see tests/test_oracle_*.py).
"""
