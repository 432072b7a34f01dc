"""CPU FP64 oracle for MPS time evolution of the ab-initio electronic Hamiltonian.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here, and nothing here
imports the product.

Contents (each function cites the passage of Frahm & Pfannkuche, arXiv:1902.08489,
that it follows):
  fci        -- occupation-number (full CI) representation, Eq. (fci); the Hamiltonian
                of Eq. (hamil) built by applying second-quantised operators with
                Jordan-Wigner signs; observables.
  slater     -- Slater-Condon matrix elements between determinants (independent of fci).
  propagate  -- exact exp(-iHt) of Eq. (time_evo_opera), the RK4 map (the RK4 stage
                definitions and Eq. (rk_add)) and the Krylov map of Eqs. (kry_non, kry_orth,
                krylov_evo).
  mps        -- dense MPS with (N_up, N_dn) bond labels, Eq. (mps); sequential-SVD
                decomposition; truncation to the D largest singular values; the
                variational two-site fit of Eq. (add_min) computed by projection; RK4 and
                Krylov drivers built from it.
  ordering   -- Fiedler ordering of the orbitals (H2O section) and the relabelling of the
                integrals.
"""
