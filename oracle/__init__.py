"""CPU FP64 oracle for the exact-diagonalisation hot path (TEST INFRASTRUCTURE).

This package is the plain, slow, obviously-correct reference that the HIP path is
checked against.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (no kernels, headers, tables or
helpers); only the seeded input dictionaries come from a common generator,
which holds none of the method's arithmetic.

Modules
  fock      -- sector basis (the build_sector listing, Sec. 6 "Sector
               construction"), fermionic signs (Sec. 2.3), the explicit sector
               Hamiltonian built on full 2Ns-bit strings (eq. Ham1), sampled rows
               of H.v for sectors too large to store.
  kron      -- the per-spin operators of the decomposition (eq. Hdecomp /
               Hbuild) as SciPy sparse matrices: a second oracle form for large
               sectors, pinned to the explicit H.
  jw        -- Jordan-Wigner Fock-space operators for tiny systems: an
               independent construction of H used to pin ``fock``.
  spectra   -- eigen-solvers: dense eigh, Lanczos with full re-orthogonalisation,
               ARPACK cross-check, the plain three-term recurrence (Sec. 6
               "Diagonalization") and the tridiagonal eigenproblem.
  green     -- impurity Green's function: exact Lehmann sum (eq. KLgf) and the
               Krylov approximation in spectral form.
  closed    -- closed forms that pin the above: non-interacting (U=0) energy and
               G, atomic-limit (V=0) energy.
  rng       -- SplitMix64 counter-based start vector (published definition).

Parity status: every function is pinned by a test in ``tests/test_oracle_*.py``
except the FP32 precision-mode error, which the paper does not fix (parity
unpinned; it is reported, not gated).
"""
