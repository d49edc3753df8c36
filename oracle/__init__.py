"""CPU oracle for the semi-implicit Fourier-spectral (FS) phase-field step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
FP64 NumPy statement of what the method computes (Boccardo et al.,
"Efficiency and accuracy of GPU-parallelized Fourier spectral methods for
solving phase-field models", arXiv:2306.04322).  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its Python binding) never imports,
links or calls anything in here, and this package imports nothing from the
product path: the two share no code.

Modules
  fft         own iterative radix-2 FFT and a brute-force O(N^2) DFT
  freeenergy  chemical free energies (paper's f_chem, Landau polynomial),
              their first derivatives and Hessians
  kspace      squared frequency |xi|^2 per Eq. (16)/(19), and the FS-FD
              symbols of Eq. (17)/(18)/(20)/(21)
  fs          the FS time step of Algorithm 1 / Eq. (10)-(15)
  fd          the explicit finite-difference comparison step (Sec. 2.2)
  energy      total free energy Eq. (1) and mass
  adjoint     discrete adjoint of the FS step and the parameter gradients
  stability   linearised per-mode stability bounds of both schemes

Every array is float64 (complex128 in k-space).  Fields are stacked as
(F, Ny, Nx) in 2D and (F, Nz, Ny, Nx) in 3D, x fastest, c first then
eta_1..eta_p.  A configuration is a plain dict (see `config_fields`).
"""

from . import fft, freeenergy, kspace, fs, fd, energy, adjoint, stability  # noqa: F401

__all__ = ["fft", "freeenergy", "kspace", "fs", "fd", "energy", "adjoint",
           "stability"]
