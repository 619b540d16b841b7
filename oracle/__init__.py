"""CPU FP64 oracle for the two-site DMRG effective-Hamiltonian path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports it, and this package
never imports the product: the two share nothing but the seeded input
generator in `synth`, which holds no effective-Hamiltonian arithmetic.

Everything here is plain and slow on purpose: Python loops over terms and
blocks with numpy matmuls in float64, dense `eigh`/`svd` from LAPACK, and
Fock-space operators built bit by bit.  Each function cites the part of
the paper (Menczer et al., arXiv:2407.07411) or the textbook definition
it follows.
"""
