"""FP64 CPU oracle for the nullspace-free Maxwell eigenproblem on Bravais lattices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP implementation.

Paper: Huang, Li, Li, Lin, Lin, Tian, "Eigenvalue Problems of Discrete Curl
Operators on Various Lattices for Simulating Three Dimensional Photonic
Crystals" (arXiv:1806.10284).

Modules
-------
geometry   Section 2.2: rotated/corrected lattice vectors, grid offsets m, mesh sizes.
curl       Section 3: explicit sparse Yee curl C with quasi-periodic wraps, A = C*C, B.
paper_forms  Section 3.1 / Theorems 4.1-4.4 transcribed as printed (used only as pins).
spectral   Section 4.2: the unitary Fourier basis T, the diagonals Lambda_1..3,
           and T q / T* p by the factored DFTs of Algorithms 5.1 / 5.2.
nfsep      Section 5.1-5.2: the mixing Q_r Sigma_r, the NFSEP operator A_r (Theorem 5.2).
solve      Smallest positive eigenvalues of A x = lambda B x (dense or sparse).
grad       Derivative of an eigenvalue with respect to the diagonal of B.

All arithmetic is float64 / complex128.
"""
