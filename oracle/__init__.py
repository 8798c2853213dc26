"""FP64 CPU oracle for the FFT-based Galerkin method with guaranteed bounds.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this package; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It is written for clarity, not speed: plain NumPy in
float64/complex128, full (non-Hermitian-reduced) spectra, full d x d
coefficient matrices, Hestenes-Stiefel CG, and a dense direct solver for tiny
grids.  It shares no code with the HIP path; the only common module is the
seeded geometry generator ``homgen``.

Modules
  spectral      index sets Z_N, DFT conventions, Helmholtz projections (Sec. 2.3, 4)
  coefficients  Fourier coefficients of matrix-inclusion and pixel media and the
                coefficient on the doubled grid (Sec. 6, Lemma on double-grid
                quadrature, Lemma on matrix-inclusion composites, Remark on
                inclusion topologies)
  galerkin      Galerkin operator without numerical integration ("Ga"), CG,
                guaranteed bounds (Sec. 3.3, 6, 7)
  dense         fully populated Fourier-Galerkin matrix (Lemma Ga_full)
  gani          Galerkin with numerical integration, the paper's Algorithm (Sec. 5, 7.2)
  unet          FP64 reference of the surrogate network (forward/backward)

Parity status: every function here is pinned by tests under tests/ against
closed forms, invariants, an independent dense formulation or brute force;
see the test names referenced in each module header.
"""
