"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/aparareal.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os

import pytest

from paper_1303_6615_amd import binding
from paper_1303_6615_amd.build import LIB_PATH


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB_PATH):
        pytest.fail("libaparareal.so not built (run python -m paper_1303_6615_amd.build)")
    return binding.lib()


def test_header_declares_the_boundary():
    syms = binding.header_symbols()
    for name in ("aparareal_create", "aparareal_destroy", "aparareal_last_error", "aparareal_nonlinear",
                 "aparareal_fine_batch", "aparareal_average", "aparareal_coarse", "aparareal_solve"):
        assert name in syms


def test_library_exports_every_declared_symbol(L):
    for name in binding.header_symbols():
        assert hasattr(L, name), name


@pytest.mark.parametrize("args", [(100, 0.01, 1.0, 0.0), (32, 0.01, 1.0, 0.0), (4096, 0.01, 1.0, 0.0),
                                  (256, 0.0, 1.0, 0.0), (256, 0.01, -1.0, 0.0), (256, 0.01, 1.0, -1e-3),
                                  (256, float("nan"), 1.0, 0.0)])
def test_create_rejects_bad_parameters(L, args):
    assert not L.aparareal_create(*args)
    assert b"" != L.aparareal_last_error()


def test_calls_reject_null_context(L):
    assert L.aparareal_fine_batch(None, None, None, 1, 0.1, 1, 0, None) == -1
    assert L.aparareal_solve(None, None, None, None, None, None) == -1
    assert L.aparareal_destroy(None) == -1
    assert b"null context" in L.aparareal_last_error()


def test_solve_params_layout_matches_header():
    # T, slices, K, dt_fine, M_avg, T0, tol, precision
    names = [f[0] for f in binding.SolveParams._fields_]
    assert names == ["T", "slices", "K", "dt_fine", "M_avg", "T0", "tol", "precision"]
    assert ctypes.sizeof(binding.SolveParams) == 56
