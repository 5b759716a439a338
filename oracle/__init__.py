"""FP64 CPU oracle for the direct inverse NFFT (Kircheis & Potts, "Direct inversion of the
nonequispaced fast Fourier transform").

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
tables or constants with the HIP path: every quantity here is recomputed from the paper's
definitions in plain NumPy (float64 / complex128).

Modules
  kb       Kaiser-Bessel window, its Fourier transform and derivative (Remark 2.1 names the
           window family without a formula; the reading used is stated in `kb`).
  direct   the exact sums (1.1)/(1.2)/(2.1) and the dense matrix A (1.3).
  nfft     the NFFT A ~ B F D (2.4)-(2.6) and the adjoint D* F* B* (2.8), dense factors.
  bopt     Algorithm 3.17: the per-grid-index least-squares problems (3.29)-(3.31), three
           independent routes (explicit L_l, reduced, Gram closed form), B_opt composition,
           the modified adjoint (3.32) and its adjoint (Remark 3.24).
  lagrange the M = N Lagrange-interpolation inverse (3.4)-(3.5), evaluated directly.
  grad     gradients of the NFFT with respect to the nodes (window derivative).
"""
from . import kb, direct, nfft, bopt, lagrange, grad  # noqa: F401
