"""Plain, slow, FP64 CPU checker for the fine-mesh correction step of the
multilevel-correction adaptive FEM for the Kohn-Sham equation (Hu, Xie, Xu).

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library imports, links or calls
this package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do. It shares no code with the library: it reads the same seeded
inputs (``inputs/``) and recomputes everything from the paper's definitions
with NumPy/SciPy (sparse assembly, ``splu``, dense ``eigh``).

Modules
  fem        P1 spaces, the 4-point quadrature, assembly, prolongation
  fem2       P2 spaces (the quadratic extension), the 27-point conical rule
  xc         LDA (Slater + PZ81) and X-alpha from their energy densities
  potentials external potentials
  hartree    multipole Dirichlet data and the Poisson solve
  mlc        one outer step of Algorithm 1 (steps 5-7) with Algorithm 2
  decomp     the precomputed pieces of Algorithm 3, checked against mlc
  scf        Algorithm 1 step 1 (coarse SCF) and a dense fine SCF
  pcg        Jacobi-preconditioned CG (for the CPU-baseline timing)
"""
