"""Functions of the per-wavenumber 3x3 linear operator.

Sec. 6.1 states that L acting on exp(ikx) r_k^alpha gives i omega_k^alpha
times the same, with omega_k^alpha = alpha*sqrt(1 + k^2/F), alpha in {-1,0,1},
so exp(tau L) is diagonal in that eigenbasis (reading: the printed modal
formula omits tau in the exponent; it is exp(i omega tau)).  The symbol L_k is
skew-Hermitian, so i L_k is Hermitian and has a unitary eigendecomposition;
for A_k = -L_k/eps + D_k (D_k a scalar) every analytic f satisfies

    f(c A_k) = V diag(f(c * lambda_j)) V^H,   lambda_j = d_k + i eta_j / eps,

where i L_k = V diag(eta) V^H.  Here V comes from LAPACK (numpy.linalg.eigh,
a library step) and the scalar functions exp and phi_j are evaluated with
mpmath at 60 significant digits, then rounded once to complex128.

phi_0(z) = exp(z), phi_j(z) = (exp(z) - sum_{i<j} z^i/i!)/z^j = sum_{i>=0} z^i/(i+j)!
(the Taylor sum is used for |z| < 1, the closed quotient otherwise).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

from .spectral import L_symbol, D_symbol

_DPS = 60


def _phi_mp(j: int, z):
    """phi_j(z) in mpmath at the working precision (z an mpc)."""
    if j == 0:
        return mp.exp(z)
    if abs(z) < 1:
        term = mp.mpf(1) / mp.factorial(j)
        total = term
        i = 0
        while True:
            i += 1
            term = term * z / (i + j)
            total += term
            if abs(term) < mp.mpf(10) ** (-_DPS - 5):
                return total
    acc = mp.exp(z)
    for i in range(j):
        acc -= z ** i / mp.factorial(i)
    return acc / z ** j


def _eig_iL(nx: int, F: float):
    """Unitary eigendecomposition of i*L_k for every k: (eta [K+1,3], V [K+1,3,3])."""
    iL = 1j * L_symbol(nx, F)
    eta, V = np.linalg.eigh(iL)
    return eta, V


def _assemble(V: np.ndarray, diag: np.ndarray) -> np.ndarray:
    """V diag(d) V^H for stacks [K+1,3,3] and [K+1,3]."""
    return np.einsum("kij,kj,klj->kil", V, diag, V.conj())


@lru_cache(maxsize=64)
def etdrk4_coefficients(nx: int, eps: float, F: float, nu: float, h: float):
    """Cox-Matthews ETDRK4 coefficient matrices for step h, per wavenumber.

    Returns a dict of complex [Nx/2+1, 3, 3] arrays (the same for all
    retained and non-retained k; only k <= Kd is ever used):

      E  = exp(hA),   E2 = exp(hA/2),   Q = (h/2) phi_1(hA/2),
      f1 = h (phi_1 - 3 phi_2 + 4 phi_3)(hA),
      f2 = h (phi_2 - 2 phi_3)(hA),
      f3 = h (-phi_2 + 4 phi_3)(hA).

    These are the published ETDRK4 weights rewritten with phi-functions; at
    z = 0 they reduce to the classical RK4 weights h/6, h/3 (for 2 f2), h/6.
    """
    eta, V = _eig_iL(nx, F)
    d = D_symbol(nx, nu)
    names = ("E", "E2", "Q", "f1", "f2", "f3")
    diag = {n: np.zeros(eta.shape, dtype=np.complex128) for n in names}
    with mp.workdps(_DPS):
        hh = mp.mpf(h)
        for kk in range(eta.shape[0]):
            for j in range(3):
                lam = mp.mpc(d[kk], 0) + mp.mpc(0, eta[kk, j]) / mp.mpf(eps)
                z = hh * lam
                zh = z / 2
                p1, p2, p3 = _phi_mp(1, z), _phi_mp(2, z), _phi_mp(3, z)
                vals = {
                    "E": mp.exp(z),
                    "E2": mp.exp(zh),
                    "Q": hh / 2 * _phi_mp(1, zh),
                    "f1": hh * (p1 - 3 * p2 + 4 * p3),
                    "f2": hh * (p2 - 2 * p3),
                    "f3": hh * (-p2 + 4 * p3),
                }
                for n in names:
                    diag[n][kk, j] = complex(vals[n])
    return {n: _assemble(V, diag[n]) for n in names}


def fast_rotation(nx: int, F: float, s) -> np.ndarray:
    """exp(s L_k) for every k; s scalar -> [K+1,3,3], s array [M] -> [M,K+1,3,3].

    In the eigenbasis L_k = V diag(-i eta) V^H, so exp(sL) = V diag(exp(-i eta s)) V^H."""
    eta, V = _eig_iL(nx, F)
    s_arr = np.atleast_1d(np.asarray(s, dtype=np.float64))
    phase = np.exp(-1j * eta[None, :, :] * s_arr[:, None, None])
    out = np.einsum("kij,mkj,klj->mkil", V, phase, V.conj())
    return out[0] if np.ndim(s) == 0 else out


def linear_propagator(nx: int, eps: float, F: float, nu: float, t: float) -> np.ndarray:
    """exp(t A_k), A_k = -L_k/eps + D_k, for every k: [K+1,3,3] (exact linear flow)."""
    eta, V = _eig_iL(nx, F)
    d = D_symbol(nx, nu)
    lam = d[:, None] + 1j * eta / eps
    return _assemble(V, np.exp(t * lam))


def apply(M: np.ndarray, uh: np.ndarray) -> np.ndarray:
    """Apply per-wavenumber 3x3 matrices [K+1,3,3] to states [..., 3, K+1]."""
    return np.einsum("kij,...jk->...ik", M, uh)
