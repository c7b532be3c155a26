"""CPU oracle for FIND selected inversion -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct complex128 implementations of what the GPU
library computes: diag(G), diag(G<), and the nearest-neighbour entries of G and
G< with the bond currents, for A = E*I - H - Sigma_L - Sigma_R on an Nx x Ny
mesh (paper, Sec. 1: A = H_0 + Sigma^r, G^r = A^{-1}, G< = G^r Sigma [G^r]^dagger;
Sec. 3.2 for the off-diagonal entries used for current density).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import anything from here.  Nothing in the product package imports
this package, and this package imports nothing from the product except the
seeded input generators (``paper_1104_0623_amd.inputs``), which hold none of
the method's arithmetic.

Modules:
  dense        -- definition written out: dense A, LAPACK inverse, G Sigma< G^dagger.
  rgf          -- an independent block-tridiagonal (recursive Green's function) sweep.
  exact        -- exact Gaussian-rational brute force on tiny meshes (pure Python).
  closed_forms -- analytic clean-ribbon / 1D-chain Green's functions and mode counts.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against the
paper's identities, closed forms, or brute force; none is marked
"parity unpinned".
"""
