"""CPU oracle for Multigrid Assisted Reanalysis (MGAR) heat-conduction topology optimisation.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 NumPy/SciPy
statement of what the GPU path computes. It is imported only by the test
suite, by the smoke check and by the benchmark's CPU-baseline leg. The GPU
library never calls it and shares no code with it; the two meet only through
the seeded inputs in ``workloads``.

Modules
-------
fe       grid numbering, element conductivity matrix (Eq 2-3), load vector,
         SIMP interpolation (Eq 4), assembled sparse K
mg       geometric multigrid hierarchy and the V-cycle (Sec. 2.2, Table 1)
solvers  MGCG (PCG preconditioned by one V-cycle) and MGAR reanalysis
         (Eq 12-21, Eq 28, Sec. 3.1); exact sparse direct reference
topopt   density filter (Eq 6-8), compliance and sensitivities (Eq 5, 9-11),
         optimality-criteria update, and the optimisation loop (Fig. 5 flow)
unet     NumPy reference for the learned-seed U-Net on the element grid, with
         optional BF16 rounding at the points where the GPU stores BF16

Every function cites the passage of the paper it follows. Readings of the
paper where it is silent or ambiguous are stated where they are used.
"""
