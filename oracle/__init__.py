"""CPU reference implementation (the oracle) of the two-grid sweeping
preconditioner of Stolk, "An improved sweeping domain decomposition
preconditioner for the Helmholtz equation" (arXiv 1412.0464).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Everything is plain NumPy/SciPy in complex128 and follows the paper's
definitions step by step, without blocking, fusion or reordering:

* ``discretization`` - PML stretching (Sec. 2.1), the 5-point PML finite
  difference operator (Sec. 4, eq. define_pml_fd) and the finite-element form
  of the compact 9-point operator with optimized coefficients (App. A); the
  3-D 7-point operator and the 27-point finite-element form (eq.
  define_H_FE, eq. def_IJ_opt, Table (b)).
* ``twogrid``  - PML-aware coarsening, tent prolongation P and R = P^T, the
  omega-Jacobi two-grid cycle with an inexact coarse solve (Sec. 4).
* ``dd``       - slab subdomains, discrete transmission T and T-tilde, the
  helper procedures and the UD / X sweeps (Sec. 2.2, Tables 2 and 3).
* ``krylov``   - right-preconditioned FGMRES and GMRES.
* ``problem``  - a setup/solve driver mirroring the GPU library's calls.
* ``problem3d`` - the same in three dimensions: 7-point PML finite
  differences on the fine level, the 27-point finite-element form of
  eq. define_H_FE with Table (b) on the coarse level, slabs of x layers.

It shares no code with the GPU library; only the seeded input generators in
``synth/`` serve both.
"""
