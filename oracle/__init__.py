"""Plain, slow CPU reference (float64 NumPy) of the AMR MHD hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library; the two meet only through the seeded inputs of ``workloads``.

Modules
  mhd    one ghost-padded patch advanced by one substep (MUSCL-Hancock
         predictor, HLLD fluxes, constrained-transport EMFs), CFL signal speed
  mhd1d  the same scheme restricted to one dimension (cell-centred B), used
         to pin the corner-transport/EMF choice by dimensional reduction
  amr    the patch hierarchy: nesting checks, same-level ghost maps,
         prolongation, restriction, flux/EMF registers and corrections,
         same-level synchronisation, the recursive level driver, CFL time
         step and conservation sums
  regrid refinement flags, clustering of flagged cells into new patches,
         and the initialisation of new patches from old ones and the parent
"""
