"""CPU FP64 oracle for the time-step-targeting DMRG hot path (test infrastructure only).

This package is the slow, plain reference that the HIP library is checked against.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it; the library
and its Python binding never do, and nothing here calls the library.

Modules
  ed            exact diagonalisation of the Hubbard model in a bit-string Fock basis
  closed_forms  non-interacting (U = 0) closed forms: tight-binding modes, App. A, App. B
  matvec        H_sb . psi, as the dense-halves definition and per symmetry block
  krylov        Lanczos basis started from phi, exp(-i tau T) and the Krylov step (Sec. II.A,
                Sec. II.C), time-step-targeting targets and weights (Sec. II.B, II.C)

Parity pins (what fixes each function independently of itself) are listed per module.
"""
