"""Plain FP64 CPU oracle for the Galerkin integral-equation solver of
Kruglyakov & Bloshanskaya (arXiv:1512.06126).

TEST INFRASTRUCTURE ONLY.  This package is imported by tests/, by the smoke
check in __graft_entry__.py and by the CPU-baseline leg of bench.py, and by
nothing else.  It shares no code with the HIP library (paper_1512_06126_amd):
neither imports the other.  The only common inputs come from giem_synth, which
holds seeded generators and no arithmetic of the method.

Every function is written from the paper's definitions and is deliberately
slow and direct: dense assembly of the 3N x 3N system, O(N^2) products, LU
solves, per-lambda boundary-value problems for the layered-media fundamental
functions, brute-force quadrature for the Galerkin coefficients.

Modules:
  packed        unpacking of the symmetry-packed table (Sect. 3.1, Lemmas 1-2)
  dense         system matrix A = S + R1 B R2, direct apply, LU solve (Sect. 2.2)
  normal_field  1-D plane-wave normal field of the layered background (Sect. 2.1)
  fundamental   U_1, U_sigma of Appendix B as two-point boundary-value problems
  vertical      cell-pair vertical integrals used by the coefficient tables
  hankel        Hankel transforms by partition and extrapolation
  tables        Galerkin coefficients B_n^m for all signed offsets (App. A-C)
  wholespace    closed-form whole-space Green's tensor tables (App. A, g = 0)
  fftpath       the three-step FFT apply done with scipy.fft (CPU baseline)
  fields        surface fields and impedance (Sect. 2.2 field recovery, Sect. 4)
"""
