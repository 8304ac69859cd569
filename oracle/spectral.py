"""Fourier pseudo-spectral setting of the 1D rotating shallow water system.

Sec. 6.1 (eq. RSW equations and the operator table below it) defines, for
u = (v1, v2, h) on the periodic interval [0, 2*pi):

    du/dt + (1/eps) L u = N(u) + D u

    L = [[0, -1, F^{-1/2} d/dx], [1, 0, 0], [F^{-1/2} d/dx, 0, 0]]
    D = hyperviscosity (reading: symbol -nu k^4, i.e. D = -nu d^4/dx^4, since
        the printed +mu d^4/dx^4 would amplify high wavenumbers, contrary to
        the stated purpose of damping them)
    N(u) = -(v1 dv1/dx, v1 dv2/dx, d(h v1)/dx)   (reading: the sign follows the
        PDE, where these terms sit on the left-hand side; the operator table
        prints them without the minus)

The paper does not state the grid, the transform or the dealiasing (it only
says the periodic problem is treated in Fourier space).  Readings:

  * grid x_j = 2*pi*j/Nx, j = 0..Nx-1;
  * forward transform  uh_k = (1/Nx) sum_j u_j exp(-i k x_j), k = 0..Nx/2
    (Hermitian half; negative k by conjugate symmetry);
  * inverse            u_j = sum_k uh_k exp(i k x_j);
  * 2/3 rule: keep |k| <= Kd = floor(Nx/3) (quadratic products are then alias
    free), states live in that band and every N evaluation is projected onto
    it, so the Nyquist mode is always zero.

Arrays: a state is complex [..., 3, Nx//2+1] (fields v1, v2, h last-but-one),
a physical field is real [..., 3, Nx].  numpy's FFT is used as a library step.
"""
import numpy as np


def dealias_cutoff(nx: int) -> int:
    """Largest retained wavenumber Kd = floor(Nx/3) (2/3 rule, reading above)."""
    return nx // 3


def wavenumbers(nx: int) -> np.ndarray:
    """k = 0..Nx/2 as float64."""
    return np.arange(nx // 2 + 1, dtype=np.float64)


def to_spectral(u: np.ndarray) -> np.ndarray:
    """Physical real [..., Nx] -> spectral [..., Nx/2+1], 1/Nx normalisation."""
    nx = u.shape[-1]
    return np.fft.rfft(u, axis=-1) / nx


def to_physical(uh: np.ndarray, nx: int) -> np.ndarray:
    """Spectral [..., Nx/2+1] -> physical real [..., Nx] (unnormalised sum)."""
    return np.fft.irfft(uh * nx, n=nx, axis=-1)


def project(uh: np.ndarray, nx: int) -> np.ndarray:
    """Zero every mode with k > Kd (2/3-rule band)."""
    out = np.array(uh, dtype=np.complex128, copy=True)
    out[..., dealias_cutoff(nx) + 1:] = 0.0
    return out


def L_symbol(nx: int, F: float) -> np.ndarray:
    """Fourier symbol L_k of the fast operator, complex [Nx/2+1, 3, 3].

    d/dx acts as multiplication by i k on exp(i k x) (Sec. 6.1)."""
    k = wavenumbers(nx)
    a = 1j * k / np.sqrt(F)
    Lk = np.zeros((k.size, 3, 3), dtype=np.complex128)
    Lk[:, 0, 1] = -1.0
    Lk[:, 0, 2] = a
    Lk[:, 1, 0] = 1.0
    Lk[:, 2, 0] = a
    return Lk


def D_symbol(nx: int, nu: float) -> np.ndarray:
    """Scalar hyperviscosity symbol -nu k^4 per wavenumber (reading above)."""
    k = wavenumbers(nx)
    return -nu * k ** 4


def nonlinear(uh: np.ndarray, nx: int) -> np.ndarray:
    """Dealiased N(u) in spectral space, [..., 3, Nx/2+1] -> same.

    N(u) = -(d/dx(v1^2/2), v1 dv2/dx, d/dx(h v1)): the first component is the
    paper's v1 dv1/dx written in conservative form (identical for smooth
    fields; with the 2/3 rule both forms give the same projected result).
    Products are formed pointwise on the grid, transformed back, multiplied by
    i k where a derivative is taken, and projected onto the retained band."""
    k = wavenumbers(nx)
    ik = 1j * k
    uh = project(uh, nx)
    v1 = to_physical(uh[..., 0, :], nx)
    v2x = to_physical(ik * uh[..., 1, :], nx)
    h = to_physical(uh[..., 2, :], nx)
    p1 = to_spectral(0.5 * v1 * v1)
    p2 = to_spectral(v1 * v2x)
    p3 = to_spectral(h * v1)
    out = np.stack([-ik * p1, -p2, -ik * p3], axis=-2)
    return project(out, nx)


def nonlinear_physical(u: np.ndarray) -> np.ndarray:
    """N(u) for physical input [..., 3, Nx]: project u onto the band, evaluate
    the dealiased N and return it on the grid."""
    nx = u.shape[-1]
    return to_physical(nonlinear(project(to_spectral(u), nx), nx), nx)


def l2_norm(uh: np.ndarray, nx: int) -> np.ndarray:
    """Discrete L2 norm over all 3*Nx grid values, sqrt(sum_j |u_j|^2), of a
    spectral state [..., 3, Nx/2+1] (evaluated on the grid)."""
    u = to_physical(uh, nx)
    return np.sqrt(np.sum(u * u, axis=(-2, -1)))
