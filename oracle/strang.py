"""Strang-splitting propagator (Alg. 3) and the standard parareal coarse step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One step of size h of u' = A u + N(u), A = -L/eps + D (exact linear part):
    v = e^{(h/2) A} u                       (half step of the linear flow)
    v = v + h N(v + (h/2) N(v))             (midpoint step of the nonlinear flow)
    u+ = e^{(h/2) A} v                      (half step of the linear flow)
Readings: the exponent of the linear half steps is (h/2)(-L/eps + D), the
sign of eq. full eqn; the nonlinear stage printed in Alg. 3 (v <- N(v);
v <- N(u_m + (h/2) v)) lacks the update and starts from u_m, and is read as
the midpoint rule started from the state after the first half step, as in
the coarse step of Alg. 2.

Standard parareal (the paper's comparison in Sec. 6.2) uses this integrator
for the coarse solver with one step per slice, and as the fine solver.
"""
import numpy as np

from .matfun import apply, linear_propagator
from .spectral import nonlinear, project


def strang_propagate(uh: np.ndarray, nx: int, eps: float, F: float, nu: float,
                     dT: float, steps: int, with_nonlinear: bool = True) -> np.ndarray:
    """Advance spectral states [..., 3, Nx/2+1] over dT with `steps` Strang steps."""
    h = dT / steps
    half = linear_propagator(nx, float(eps), float(F), float(nu), 0.5 * h)

    def N(v):
        return nonlinear(v, nx) if with_nonlinear else np.zeros_like(v)

    u = project(uh, nx)
    for _ in range(steps):
        v = apply(half, u)
        v = v + h * N(v + (0.5 * h) * N(v))
        u = apply(half, v)
    return u
