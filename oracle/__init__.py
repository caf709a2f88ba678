"""FP64 CPU oracle for the singularity-subtracted fractional Laplacian solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything in this package;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, tables or constants with the GPU
path: every formula here is written out again from the paper (Minden & Ying,
"A simple solver for the fractional Laplacian in multiple dimensions").

Modules
-------
constants  C_{alpha,d}, the lattice sum A_1 (Ewald split), A_2, A_3, the
           window W (Sec. 2.5-2.7, eqs. int1constants, a3, window)
operator   weights w_m, the dense BTTB matrix M, the circulant embedding and
           its symbol, naive-DFT application (Sec. 3.1, eqs. linearelliptic,
           matelliptic, "Forward operator and application with FFT")
precond    the finite-difference Laplacian preconditioner C h^d L and its
           exact inverse by dense sine transforms (Sec. 3.1, "Preconditioning")
krylov     CG / PCG, flexible CG, theta-scheme time stepping (Sec. 3.1, 3.2)
unet       reference forward/backward of the learned preconditioner network
           (not in the paper; parity pinned by finite differences)

Every function is plain and slow on purpose.  Floating point is float64.
"""
