"""Planted mistakes in the oracle are caught by its pins (CPU only).

Each case plants one plausible mistake in the oracle (a flipped sign, a
transposed operand, a dropped term, a wrong normalisation) by replacing a
function in the oracle's own module namespace for the duration of the test,
then runs one of the pins of tests/test_oracle_pins.py and requires it to
fail.  This shows the pins would see such mistakes; nothing here changes the
oracle itself.
"""
import numpy as np
import pytest

import oracle
import oracle.etdrk4
import oracle.hmm
import oracle.matfun
import oracle.spectral
import tests.test_oracle_pins as pins


def _clear_caches():
    oracle.matfun.etdrk4_coefficients.cache_clear()


@pytest.fixture(autouse=True)
def _fresh_caches():
    _clear_caches()
    yield
    _clear_caches()


def _nonlinear_sign(mp):
    orig = oracle.spectral.nonlinear
    mp.setattr(oracle, "nonlinear", lambda uh, nx: -orig(uh, nx))


def _nonlinear_transposed(mp):
    # v1 and v2 exchanged before the products (a transposed operand)
    orig = oracle.spectral.nonlinear
    mp.setattr(oracle, "nonlinear", lambda uh, nx: orig(uh[..., [1, 0, 2], :], nx))


def _no_dealiasing(mp):
    orig = oracle.spectral.nonlinear
    mp.setattr(oracle.spectral, "project", lambda uh, nx: uh)
    mp.setattr(oracle, "nonlinear", orig)


def _coefficients(mutate):
    orig = oracle.matfun.etdrk4_coefficients

    def bad(nx, eps, F, nu, h):
        co = dict(orig(nx, eps, F, nu, h))
        mutate(co)
        return co
    return bad


def _etdrk4_drop_f3(mp):
    def m(co):
        co["f3"] = np.zeros_like(co["f3"])
    mp.setattr(oracle.etdrk4, "etdrk4_coefficients", _coefficients(m))


def _etdrk4_swap_f1_f3(mp):
    def m(co):
        co["f1"], co["f3"] = co["f3"], co["f1"]
    mp.setattr(oracle.etdrk4, "etdrk4_coefficients", _coefficients(m))


def _hyperviscosity_sign(mp):
    orig = oracle.spectral.D_symbol
    mp.setattr(oracle.matfun, "D_symbol", lambda nx, nu: -orig(nx, nu))


def _rotation_direction(mp):
    orig = oracle.matfun.fast_rotation
    mp.setattr(oracle.hmm, "fast_rotation", lambda nx, F, s: orig(nx, F, -np.asarray(s)))


def _weights_unnormalised(mp):
    orig = oracle.hmm.average_weights
    mp.setattr(oracle.hmm, "average_weights", lambda M: orig(M) * M)


def _coarse_without_dissipation(mp):
    orig = oracle.spectral.D_symbol
    mp.setattr(oracle.hmm, "D_symbol", lambda nx, nu: 0.0 * orig(nx, nu))


CASES = [
    ("sign of N", _nonlinear_sign, lambda: pins.test_nonlinear_matches_galerkin_convolution(16)),
    ("v1 and v2 transposed in N", _nonlinear_transposed, lambda: pins.test_nonlinear_matches_galerkin_convolution(16)),
    ("2/3 rule dropped", _no_dealiasing, pins.test_nonlinear_dealiasing_band),
    ("ETDRK4 f3 term dropped", _etdrk4_drop_f3, pins.test_etdrk4_fourth_order),
    ("ETDRK4 f1 and f3 transposed", _etdrk4_swap_f1_f3, pins.test_etdrk4_fourth_order),
    ("hyperviscosity sign", _hyperviscosity_sign,
     lambda: pins.test_etdrk4_coefficients_match_block_expm(0.1, 3e-5, 0.002)),
    ("rotation direction of the coarse step", _rotation_direction, pins.test_linear_case_fine_coarse_parareal_exact),
    ("average weights without 1/M", _weights_unnormalised, pins.test_average_short_window_is_weighted_nonlinear),
    ("coarse step without its dissipative half steps", _coarse_without_dissipation,
     pins.test_linear_case_fine_coarse_parareal_exact),
]


@pytest.mark.parametrize("name,plant,pin", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_fails_a_pin(monkeypatch, name, plant, pin):
    plant(monkeypatch)
    _clear_caches()
    with pytest.raises(AssertionError):
        pin()
