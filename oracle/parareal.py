"""The asymptotic parareal iteration (Sec. 3, eq. HMM parareal iteration; Alg. 4).

    U_n^0 = G(U_{n-1}^0)
    U_n^k = G(U_{n-1}^k) + Fine(U_{n-1}^{k-1}) - G(U_{n-1}^{k-1}),  k >= 1

with U_0^k = u0, G the asymptotic coarse step and Fine the ETDRK4 slice
propagator.  Readings:

  * slices n = 1..Ns on [0, T], dT = T/Ns, output U_0..U_Ns (Alg. 4's loop
    bounds 1..N-1 and its return of U_1..U_N disagree);
  * a fixed number K of iterations (the tolerance loop of Alg. 4 is the
    `tol` argument, off by default);
  * G(U_{n-1}^{k-1}) is the value computed in the previous sweep, reused, and
    the update is evaluated as Fine_old + (G_new - G_old) in FP64;
  * residual of iteration k: max_n ||U_n^k - U_n^{k-1}|| / ||U_n^k|| with the
    discrete L2 norm over all 3*Nx grid values (Alg. 4 leaves the norm open).
"""
import numpy as np

from .etdrk4 import fine_propagate
from .hmm import coarse_propagate
from .spectral import l2_norm, project, to_physical, to_spectral


def parareal_solve(u0: np.ndarray, nx: int, eps: float, F: float, nu: float,
                   T: float, Ns: int, K: int, fine_steps: int, Mbar: int,
                   T0: float, tol: float = 0.0, with_nonlinear: bool = True,
                   coarse=None, fine=None):
    """Run the iteration from the physical initial state u0 [3, Nx].

    Returns (U, resid, history): U physical [Ns+1, 3, Nx] after the last
    iteration, resid the list of residuals r^1..r^K, history the spectral
    iterates [K+1][Ns+1, 3, Nx/2+1] (for the parareal-property checks).
    `coarse`/`fine` override the propagators (test hooks)."""
    dT = T / Ns

    def G(v):
        if coarse is not None:
            return coarse(v)
        return coarse_propagate(v, nx, eps, F, nu, dT, T0, Mbar, with_nonlinear)

    def Fn(v):
        if fine is not None:
            return fine(v)
        return fine_propagate(v, nx, eps, F, nu, dT, fine_steps, with_nonlinear)

    u0h = project(to_spectral(np.asarray(u0, dtype=np.float64)), nx)
    U = np.zeros((Ns + 1,) + u0h.shape, dtype=np.complex128)
    Gold = np.zeros_like(U)
    U[0] = u0h
    for n in range(1, Ns + 1):
        Gold[n] = G(U[n - 1])
        U[n] = Gold[n]
    history = [U.copy()]
    resid = []
    for _ in range(K):
        Fold = np.zeros_like(U)
        Fold[1:] = Fn(U[:-1])                     # every slice at once (the parfor)
        Unew = np.zeros_like(U)
        Unew[0] = u0h
        for n in range(1, Ns + 1):
            g = G(Unew[n - 1])
            Unew[n] = Fold[n] + (g - Gold[n])
            Gold[n] = g
        num = l2_norm(Unew[1:] - U[1:], nx)
        den = l2_norm(Unew[1:], nx)
        resid.append(float(np.max(num / den)))
        U = Unew
        history.append(U.copy())
        if tol > 0.0 and resid[-1] <= tol:
            break
    return to_physical(U, nx), resid, history


def serial_fine(u0: np.ndarray, nx: int, eps: float, F: float, nu: float,
                T: float, Ns: int, fine_steps: int, with_nonlinear: bool = True):
    """Serial fine chain U_n* = Fine^n(u0), spectral [Ns+1, 3, Nx/2+1]."""
    dT = T / Ns
    u = project(to_spectral(np.asarray(u0, dtype=np.float64)), nx)
    out = [u]
    for _ in range(Ns):
        u = fine_propagate(u, nx, eps, F, nu, dT, fine_steps, with_nonlinear)
        out.append(u)
    return np.stack(out)
