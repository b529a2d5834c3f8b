"""CPU oracle for the LNV density-matrix hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, dense FP64 numpy/scipy implementation of what the GPU path
computes, written from Sec. II.C.2 of the paper ("Density matrix: linear
scaling"): range-truncated auxiliary matrix L, the McWeeny form
K = 3LSL - 2LSLSL, band energy E = 2 Tr[KH], electron number N = 2 Tr[KS],
their gradients with respect to the stored entries of L, and a conjugate
gradient minimisation with the electron-number constraint.

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import or run anything in this package.  It shares no code with
the HIP path (`paper_2002_07704_amd`) and neither imports the other; the only
common dependency is `lnv_workloads`, which generates seeded inputs and holds
none of the method's arithmetic.

Modules
  structure  neighbour lists (brute force), synthetic S/H, dense<->block maps
  lnv        K, E, N, G, F, dE/dS, dE/dH, cubic line coefficients, CG, exact K
  rows       the same quantities for a few sampled atom rows of a large cell
"""
