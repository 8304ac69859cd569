"""Pins of the Strang-splitting oracle (Alg. 3) and of standard parareal,
against things other than itself: the exact linear flow, an independent
high-order ODE solution (second-order convergence), the conserved mean of h
and the parareal property."""
import math

import numpy as np
import pytest

import oracle as O
from oracle.matfun import apply, linear_propagator
from oracle.strang import strang_propagate
from paper_1303_6615_amd.inputs import seeded_state


def _state(nx, seed, amp=0.1, k_ic=None):
    return O.project(O.to_spectral(seeded_state(nx, k_ic or nx // 4, seed, amplitude=amp)), nx)


def test_linear_case_is_the_exact_flow():
    # N = 0: the two half steps compose to exp(h A) per step, exactly
    nx, eps, F, nu = 32, 0.05, 1.3, 1e-4
    uh = _state(nx, 3, amp=1.0)
    got = strang_propagate(uh, nx, eps, F, nu, 0.37, 7, with_nonlinear=False)
    want = apply(linear_propagator(nx, eps, F, nu, 0.37), uh)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_second_order_convergence():
    # against ETDRK4 with a far smaller step (itself pinned to DOP853)
    nx, eps, F, nu = 32, 0.1, 1.0, 1e-4
    uh = _state(nx, 9, amp=0.1)
    dT, base = 0.1, 8          # asymptotic range (4 steps still show order 2.3)
    ref = O.fine_propagate(uh, nx, eps, F, nu, dT, 512)
    errs = [np.linalg.norm(strang_propagate(uh, nx, eps, F, nu, dT, base * m) - ref) for m in (1, 2, 4)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 <= o <= 2.2 for o in orders), orders


def test_mean_of_h_is_conserved():
    nx = 32
    uh = _state(nx, 5, amp=0.3)
    uh[2, 0] = 0.25                                  # nonzero mean height
    out = strang_propagate(uh, nx, 0.1, 1.0, 1e-3, 0.2, 9)
    assert abs(out[2, 0] - 0.25) < 1e-15


def test_zero_state_is_a_fixed_point():
    nx = 32
    z = np.zeros((3, nx // 2 + 1), dtype=np.complex128)
    assert np.all(strang_propagate(z, nx, 0.1, 1.0, 1e-3, 0.2, 3) == 0)


@pytest.mark.parametrize("K", [2, 5])
def test_standard_parareal_property(K):
    # coarse: one Strang step per slice; fine: Strang steps of dt.  After k
    # iterations the first k slices equal the serial fine chain bitwise; with
    # K = Ns + 1 the last residual is exactly zero.
    nx, eps, F, nu, T, Ns, M = 32, 0.1, 1.0, 1e-3, 0.4, 4, 10
    u0 = seeded_state(nx, 8, 12, amplitude=0.2)
    dT = T / Ns
    coarse = lambda v: strang_propagate(v, nx, eps, F, nu, dT, 1)          # noqa: E731
    fine = lambda v: strang_propagate(v, nx, eps, F, nu, dT, M)            # noqa: E731
    U, res, hist = O.parareal_solve(u0, nx, eps, F, nu, T, Ns, Ns + 1, M, 8, dT / eps, coarse=coarse, fine=fine)
    u = O.project(O.to_spectral(u0), nx)
    chain = [u]
    for _ in range(Ns):
        chain.append(fine(chain[-1]))
    for k in range(Ns + 2):
        for n in range(min(k, Ns) + 1):
            assert np.array_equal(hist[k][n], chain[n]), (k, n)
    assert res[-1] == 0.0
