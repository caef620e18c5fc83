"""CPU FP64 oracle for the local Krylov-subspace density-matrix solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg do.  It shares no code with the HIP path:
it is a plain, slow, obviously-correct NumPy restatement of what the paper
defines (Iitaka, "GPU-accelerated large-scale quantum molecular dynamics
simulation of 3-dimensional C60 polymers"):

  * model.py     -- tight-binding Hamiltonian of Eq. (1) in the sp3
                    Slater-Koster form, its radial functions and the
                    repulsive pair functional;
  * geometry.py  -- minimum-image neighbour and cutoff-sphere lists (Sec. 2,
                    the locality argument that gives O(n^3 N) cost);
  * krylov.py    -- the Krylov subspace of Eq. (4) seeded with the target
                    atom's orbitals, its orthonormal basis, and the Lanczos
                    recursion of Eqs. (6)-(9) in block form (Sec. 3);
  * tb.py        -- per-atom projected eigensolve, the occupation / global
                    chemical potential, the density matrix of Eq. (2), band
                    energy and the forces Tr[rho dH/dR] (Sec. 2);
  * exact.py     -- the O(N^3) full diagonalisation the paper contrasts the
                    method with (Sec. 2), for tiny systems;
  * timing.py    -- timing of a bounded sample of atom-solves on host cores.

Pins (what fixes this oracle independently of itself) live in
tests/test_oracle_*.py.  Parity unpinned: production-size results at finite
Krylov order r and finite cluster radius are fixed only by the definition
(the paper prints no values); they are cross-checked by two independent
basis constructions (block Arnoldi with sequential Gram-Schmidt, and the
block three-term recursion with pivoted Householder QR).
"""
