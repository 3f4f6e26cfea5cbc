"""CPU FP64 oracle for the layered-grating multi-inclusion scattering method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP
library: special functions come from SciPy (AMOS), linear algebra from
NumPy/LAPACK, and every formula is restated from the paper (Lai, Kobayashi,
Barnett, "A fast and robust solver for the scattering from a layered periodic
structure containing multi-particle inclusions").

Modules
  common      derived physical quantities, nodes, multipole helpers (sec. 2, 3)
  quadrature  zeta-corrected trapezoid rule for the log-singular self blocks (sec. 3)
  layered     the empty-structure matrix A and right-hand side f (sec. 3, eq. matA/Arhs)
  multiple    single-disk scattering matrix and the translation operator T (sec. 4)
  coupling    the coupling blocks B (layers -> inclusions) and C (inclusions -> rows) (sec. 5)
  solver      pseudo-inverse, reduced operator, LU / GMRES, Bragg amplitudes, flux (sec. 5, 6)

Every function is pinned by a CPU test against something other than itself
(closed forms, identities, special cases, brute force); see tests/test_oracle_*.py.
"""
