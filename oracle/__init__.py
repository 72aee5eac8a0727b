"""CPU FP64 oracle for the iterative Poisson / self-gravity solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library; the only module both sides use is ``workloads`` (seeded inputs).

The oracle computes the *plain definitions* that every iterative solver of the
paper converges to, written slowly and directly in float64:

* ``harmonics``  -- real orthonormal spherical harmonics and the normalised
  solid harmonics of the multipole expansion (Section 2.2).
* ``multipole``  -- outer / inner multipole moments and the ghost-zone
  potential they imply (Section 2.2, Eqs. outer_expansion .. inner_multipole).
* ``operators``  -- the discrete Laplacians (Eq. 1 with the 2nd-order 7-point
  and the 6th-order 19-point star; Eq. 2 on the log-spherical grid) and the
  residual (Section 2.1).
* ``smoothers``  -- one red-black SOR colour pass (Section 2.1.1), one
  four-colour Gauss-Seidel pass (Section 2.1.2), full-weighting restriction,
  the prolongation P = cR^T and a reference V-cycle (Section 2.1.3).
* ``direct``     -- the exact discrete solution: DST-I for the 7-point
  operator, DST-preconditioned CG for the 19-point star, per-azimuthal-mode
  sparse LU on the spherical grid, and brute-force dense solves.
* ``analytic``   -- closed-form potentials used to pin the above.

Parity status: every function is pinned by tests under ``-m "not gpu"``
except where its docstring says "parity unpinned".
"""
