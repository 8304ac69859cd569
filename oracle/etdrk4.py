"""Fine propagator: exponential time differencing RK4 (Cox & Matthews).

Sec. 6.2 uses ETDRK4 as the fine integrator (cited, formulas not printed);
every workload here steps each parareal slice with it.  For
u' = A u + N(u), step h, with the coefficient matrices of matfun:

    a  = E2 u + Q N(u)
    b  = E2 u + Q N(a)
    c  = E2 a + Q (2 N(b) - N(u))
    u+ = E u + f1 N(u) + 2 f2 (N(a) + N(b)) + f3 N(c)

The slice of length dT is covered by `steps` equal steps h = dT/steps
(reading: when dT/dt is not an integer the step count is ceil(dT/dt) and the
step is shortened to dT/steps, so it never exceeds the requested dt).
"""
import math

import numpy as np

from .matfun import apply, etdrk4_coefficients
from .spectral import nonlinear, project


def fine_step_count(dT: float, dt: float) -> int:
    """Number of fine steps per slice, ceil(dT/dt) up to a 1e-9 relative slack."""
    return max(1, int(math.ceil(dT / dt - 1e-9)))


def fine_propagate(uh: np.ndarray, nx: int, eps: float, F: float, nu: float,
                   dT: float, steps: int, with_nonlinear: bool = True) -> np.ndarray:
    """Advance spectral states [..., 3, Nx/2+1] over dT with `steps` ETDRK4 steps.

    `with_nonlinear=False` drops N (test hook for the exactly solvable linear case)."""
    h = dT / steps
    co = etdrk4_coefficients(nx, float(eps), float(F), float(nu), float(h))
    E, E2, Q, f1, f2, f3 = (co[n] for n in ("E", "E2", "Q", "f1", "f2", "f3"))

    def N(v):
        if with_nonlinear:
            return nonlinear(v, nx)
        return np.zeros_like(v)

    u = project(uh, nx)
    for _ in range(steps):
        Nu = N(u)
        E2u = apply(E2, u)
        a = E2u + apply(Q, Nu)
        Na = N(a)
        b = E2u + apply(Q, Na)
        Nb = N(b)
        c = apply(E2, a) + apply(Q, 2.0 * Nb - Nu)
        Nc = N(c)
        u = apply(E, u) + apply(f1, Nu) + 2.0 * apply(f2, Na + Nb) + apply(f3, Nc)
    return u
