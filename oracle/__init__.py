"""FP64 CPU oracle for the recursive multiscale Robin coupled method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the tests, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with
the HIP path (the two meet only at the seeded input generators in
``workloads``).

Contents, each written from the paper (Abreu et al., "Recursive
formulation and parallel implementation of multiscale mixed methods"):

* ``tpfa``       — lowest-order RT0 with a lumped velocity mass, i.e. the
                   two-point cell-centred finite-volume scheme (Section 2.1
                   and Section 4: a pressure-only linear system).
* ``decomp``     — the non-overlapping decomposition, skeleton segments of
                   size Hbar, the global normal and the Robin parameter
                   (Section 2 decomposition equations; Section 5.1 Robin
                   beta and effective-permeability equations).
* ``fine``       — O-1: the global fine-grid solve.
* ``local``      — O-2: the local Robin problems (Section 2, eq. 11.2-12.2;
                   the basis problems of Section 2.1 and the particular
                   solution of the additive split).
* ``mrcm``       — O-3: the plain non-recursive method: the interface
                   system A X = b (Section 2.2) and the final local
                   solution.
* ``monolithic`` — O-4: brute force on tiny grids, every cell pressure and
                   every interface unknown in one dense system.
* ``recursive``  — O-5: Algorithm 1 (recursive formulation, Section 3)
                   over the nested binary hierarchy.
* ``three_d``    — O-6: the three-dimensional method of the paper's
                   experiments (seven-point scheme, no z-division, Hbar_z =
                   H_z): fine solve, local problems, non-recursive MRCM and
                   a face-by-face brute force.
* ``metrics``    — norms and conservation / interface-equation residuals.
* ``cnn``        — the local-basis surrogate network (forward, loss,
                   gradients, input features) in FP64, for checking the GPU
                   training and inference kernels.

Every floating-point value is float64.  Parity status of each function is
stated in its docstring; all are pinned by the ``-m "not gpu"`` tests.
"""
