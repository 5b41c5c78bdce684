"""CPU FP64 oracle for the density-matrix approximate contraction.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only tests/, the smoke check in __graft_entry__ and the cpu_baseline leg of bench.py
use it. It shares no code with the HIP path; the only common input is the seeded
network generator in paper_2406_09769_amd.inputs, which holds no arithmetic of the
method.

Modules:
  dm      the density-matrix algorithm (Algorithm density_matrix_alg with the
          memoised density matrices of Eq. dm_cache) on a maximally unbalanced
          partition path with the MPS ansatz, plus its structural planner
  canon   the canonicalisation twin (Algorithm canonize applied to the explicit,
          untruncated boundary) that pins the approximate result
  exact   exact references: brute force, transfer matrices, Onsager
  mlp     the warm-start MLP forward/backward in numpy
"""
