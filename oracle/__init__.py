"""CPU oracle: a plain, slow, FP64 reference of the GNN-smoothed AMG solve phase.

TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library, its Python
binding) imports, links or calls this package; only the tests, the smoke check
and the CPU-baseline leg of the benchmark do. It shares no code with the GPU
path: the two meet only in the seeded input generators of ``workloads``.

Modules
-------
amg   : Ruge-Stueben setup, sparse pseudo-inverse smoother, V-cycle, coarse
        solve, stationary / iterative-refinement / flexible-CG solves.
gcin  : the GCIN coefficient predictor (forward in FP64 PyTorch CPU ops, its
        gradient by autograd).
grad  : loss of one V-cycle and its gradient w.r.t. the smoother coefficients
        by complex step and by central finite differences.

Every function cites the passage of the paper it follows. Points where the paper
is silent or ambiguous carry a "Reading:" note; the same list is kept with the
design notes of the repository.
"""
