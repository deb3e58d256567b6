"""CPU oracle for the branch-and-bound tensor network (BBTN) hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package.  It shares
no code with the GPU path (no kernels, headers, helpers or tables) and imports
nothing from it; the only common module is `instances`, which generates seeded
inputs and holds none of the method's arithmetic.

What the method computes has a plain definition (Eq. 1-2 and the MWIS
paragraph of the "Tropical Tensor Networks" section): the minimum of the
energy (or the maximum independent-set weight) over all configurations and
the number of configurations reaching it.  Branching is exact by construction
(complete and orthogonal branches, pruning of strictly suboptimal
configurations only, "Branch-and-Bound Tensor Network" section), so the
oracle needs no planner: it evaluates that definition directly.

Modules
  semiring    counting tropical algebra, exact integers (Eq. 2 and the tuple
              algebra of the counting paragraph)
  brute       brute-force enumeration over all 2^n configurations
  tm          exact transfer-matrix solvers for lattices (spin glass, KSG)
  ve          exact variable elimination on arbitrary graphs
  value       value-only checks through library routines (matching, MILP)
  device_ops  the per-kernel operations in the device encoding (max form,
              int32 values, residues modulo primes)
  crt         Chinese remaindering of residues into an exact integer
  mlp         the branching scorer's MLP, forward/backward/Adam in float64
"""
