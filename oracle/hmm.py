"""HMM time average of the nonlinear term and the asymptotic slow solver.

Sec. 2 (eq. numerical average, discretized) approximates the infinite-time
average of exp(sL) N(exp(-sL) u) by a kernel-weighted trapezoid rule,

    Nbar(u) = (1/Mbar) sum_{m=0}^{Mbar-1} rho(s_m/T0) exp(s_m L) N(exp(-s_m L) u),
    s_m = m T0 / Mbar,

with the smooth kernel rho(s) = C exp(-1/(s(1-s))) on (0,1), zero elsewhere,
C normalising its integral to one (end of Sec. 2).  Alg. 1 evaluates the
samples independently and sums them.  Readings:

  * s is fast time: it multiplies L directly, as in Alg. 1 and in the
    infinite average (the variant with s/eps in Sec. 2 is the same integral
    after a change of variables, and mixing the two would double-count eps);
  * Alg. 1's loop index j vs m and its Sum over 1..Mbar are read as the
    trapezoid sum above, including the 1/Mbar; the m = 0 term has weight
    rho(0) = 0 and is kept in the sum (it contributes exactly zero);
  * C normalises the continuous integral, so the discrete weights sum to
    slightly less than one.

Alg. 2 (asymptotic slow solver) is read as Strang splitting of the averaged
equation: a half step of the dissipative flow, one explicit midpoint step of
the averaged nonlinear flow, a second dissipative half step, then the fast
rotation back.  Readings: the printed midpoint lines overwrite the state with
the average itself and restart from u0; they are read as the standard
midpoint update w <- w + dT*Nbar(w + (dT/2)*Nbar(w)) starting from the state
after the first half step.  The final rotation is exp(-(dT/eps) L), matching
the definition of the asymptotic approximation in Sec. 3
(phi-bar_t = exp(-(t/eps)L) psi_t), which pairs with exp(+sL) N(exp(-sL) .)
inside the average; the algorithm's printed exp(+(dT/eps)L) is the
inconsistent one.  Nbar is autonomous: the window is [0, T0] at both stages.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

from .matfun import fast_rotation
from .spectral import D_symbol, nonlinear, project


@lru_cache(maxsize=1)
def rho_normaliser() -> float:
    """C = 1 / int_0^1 exp(-1/(s(1-s))) ds (mpmath quadrature, 40 digits)."""
    with mp.workdps(40):
        integral = mp.quad(lambda s: mp.exp(-1 / (s * (1 - s))), [0, 0.5, 1])
        return float(1 / integral)


def rho(s) -> np.ndarray:
    """rho(s) = C exp(-1/(s(1-s))) for 0 < s < 1, else 0 (vectorised)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    inside = (s > 0.0) & (s < 1.0)
    si = s[inside]
    out[inside] = rho_normaliser() * np.exp(-1.0 / (si * (1.0 - si)))
    return out


def average_weights(Mbar: int) -> np.ndarray:
    """Trapezoid weights rho(m/Mbar)/Mbar for m = 0..Mbar-1 (s_m/T0 = m/Mbar)."""
    return rho(np.arange(Mbar, dtype=np.float64) / Mbar) / Mbar


def sample_times(T0: float, Mbar: int) -> np.ndarray:
    """s_m = m T0 / Mbar, m = 0..Mbar-1 (fast time)."""
    return T0 * np.arange(Mbar, dtype=np.float64) / Mbar


def averaged_nonlinear(vh: np.ndarray, nx: int, F: float, T0: float, Mbar: int,
                       with_nonlinear: bool = True) -> np.ndarray:
    """Nbar(v) for spectral states [..., 3, Nx/2+1] (eq. numerical average; Alg. 1)."""
    vh = project(vh, nx)
    if not with_nonlinear:
        return np.zeros_like(vh)
    s = sample_times(T0, Mbar)
    w = average_weights(Mbar)
    back = fast_rotation(nx, F, -s)       # exp(-s_m L)  [M, K+1, 3, 3]
    fwd = fast_rotation(nx, F, s)         # exp(+s_m L)
    x = np.einsum("mkij,...jk->m...ik", back, vh)
    n = nonlinear(x, nx)
    y = np.einsum("mkij,m...jk->m...ik", fwd, n)
    return np.tensordot(w, y, axes=(0, 0))


def coarse_propagate(uh: np.ndarray, nx: int, eps: float, F: float, nu: float,
                     dT: float, T0: float, Mbar: int,
                     with_nonlinear: bool = True) -> np.ndarray:
    """One asymptotic coarse step of length dT (Alg. 2, readings in the module doc)."""
    half_diss = np.exp(D_symbol(nx, nu) * (dT / 2.0))        # exp((dT/2) D), scalar per k
    w = half_diss * project(uh, nx)
    k1 = averaged_nonlinear(w, nx, F, T0, Mbar, with_nonlinear)
    k2 = averaged_nonlinear(w + (dT / 2.0) * k1, nx, F, T0, Mbar, with_nonlinear)
    w = w + dT * k2
    w = half_diss * w
    rot = fast_rotation(nx, F, -dT / eps)                    # exp(-(dT/eps) L)
    return np.einsum("kij,...jk->...ik", rot, w)
