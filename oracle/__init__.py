"""Plain FP64 CPU oracle for the hyper-power preconditioned Stokes solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  It shares no code with ``paper_2311_06926_amd`` (the
product): no kernels, tables, helpers or constants; neither imports the
other.

Source: M.L. Mika, M.F.P. ten Eikelder, D. Schillinger, R.R. Hiemstra,
"Matrix-free polynomial preconditioning of saddle point systems using the
hyper-power method" (arXiv 2311.06926).  Every function cites the section,
equation or appendix it follows.

Modules
-------
splines     univariate B-splines (Cox--de Boor) and unit-integral M-splines
            (App. B.1, eq. ``reduction``)
matrices1d  the univariate matrices M, K, C, M^, K^, C^, N^, B^, T^
            (App. B.3, Sec. 3.3)
assemble    the saddle-point matrix by Kronecker products (Sec. 3.3) and,
            at tiny sizes, by direct 3D quadrature of the weak form
            (Sec. 3.1-3.2); right-hand sides
precond     base preconditioner P0 (Sec. 4, eq. ``blockdiagprecond``) by
            sparse LU, and the hyper-power sequences (eqs. ``Pcv``,
            ``Pcq1``, ``Pcq2``) as literal recursions
krylov      preconditioned MINRES and right-preconditioned flexible GMRES
direct      bordered direct solve with a mean-zero pressure
cases       the benchmark problem set-ups (lid-driven cavity, Sec. 5)

Parity status: every function is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, library routines, brute force or the
paper's printed numbers; none is "parity unpinned".
"""
