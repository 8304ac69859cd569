"""Plain FP64 CPU oracle for the asymptotic parareal method (Haut & Wingate).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the GPU path: its own transforms (numpy's FFT as a library
step), its own matrix functions (unitary eigendecomposition of each 3x3 Fourier
symbol plus high-precision scalar exponential/phi functions), its own averaging
and parareal driver.  Inputs come in as arrays; no random numbers are drawn here.

What each module follows:

  spectral   grid, Fourier convention, 2/3-rule dealiasing, the RSW operators
             L, D and the quadratic term N                  (Sec. 6.1, eq. RSW)
  matfun     f(hA_k) for A_k = -L_k/eps + D_k via the eigenstructure of L
             (Sec. 6.1, eigenvalues i*omega_k^alpha); scalar exp and phi_j
  etdrk4     the fine propagator: Cox-Matthews ETDRK4 (cited in Sec. 6.2)
  strang     the Strang-splitting propagator (Alg. 3), fine solver and the
             coarse solver of standard parareal
  hmm        the kernel rho, the trapezoid-rule time average of the
             nonlinear term (eq. numerical average; Alg. 1) and the
             asymptotic slow solver (Alg. 2)
  parareal   the parareal iteration (eq. HMM parareal iteration; Alg. 4)
  model      the paper's speedup estimate (eq. speedup upper bound)

Readings taken where the paper is silent, garbled or self-inconsistent are
listed in the docstrings where they are used.
Every function here is pinned by a CPU test against something other than
itself (closed forms, brute force, library routines, invariants).
"""

from .spectral import (  # noqa: F401
    dealias_cutoff, wavenumbers, to_spectral, to_physical, project,
    L_symbol, nonlinear, nonlinear_physical, l2_norm,
)
from .matfun import etdrk4_coefficients, fast_rotation, linear_propagator  # noqa: F401
from .etdrk4 import fine_propagate  # noqa: F401
from .strang import strang_propagate  # noqa: F401
from .hmm import rho, rho_normaliser, average_weights, averaged_nonlinear, coarse_propagate  # noqa: F401
from .parareal import parareal_solve, serial_fine  # noqa: F401
from .model import estimated_speedup, speedup_upper_bound  # noqa: F401
