"""MI355X-native hot path of time-step-targeting DMRG: the superblock product H_sb . psi and the
Krylov exponential exp(-i tau H) psi, behind the C ABI of libdmrgtst.so (include/dmrgtst.h).

Submodules
  inputs   seeded synthetic and exact-block workloads (no method arithmetic)
  lib      ctypes binding of the C ABI (argument marshalling only)
"""
