"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/aparareal.h declares, and rejects bad arguments before touching a device."""
import ctypes
import math
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


def _deps(job, K, groups, split):
    """Jobs that must precede `job` = (type, k, n, g) in the hand-out order."""
    t, k, n, g = job

    def step(kk, nn):            # the jobs that complete C(kk, nn)
        if kk >= 1 and nn <= kk:
            return [(4, kk, nn, 0)]
        return [(3, kk, nn, x) for x in range(groups)] if split else [(0, kk, nn, 0)]
    if t == 4:                   # exact slice: after C(k-1, n) and, for n = k, F(k-1, k)
        return step(k - 1, n) + ([(1, k - 1, n, 0)] if n == k else [])
    prev = step(k, n - 1) if n > 1 else []
    if t in (1, 2):
        return prev
    before = [(1, k - 1, n, 0)] + step(k - 1, n) if k >= 1 else []
    if t == 0:
        return prev + before
    return [(2, k, n, x) for x in range(groups)] + before     # stage 2 (any may finish the step)


@pytest.mark.parametrize("N,T,Ns,K,dt,M,split,group", [
    (64, 1.0, 16, 5, 0.0005, 16, -1, 0), (256, 2.0, 64, 8, 0.0005, 32, -1, 0),
    (256, 2.0, 64, 8, 0.0005, 32, 0, 0), (128, 0.7, 7, 3, 0.1, 2, 1, 0), (512, 1.0, 5, 0, 0.01, 8, -1, 3),
    (1024, 1.0, 256, 10, 0.0001, 64, -1, 0), (2048, 1.0, 3, 9, 1e-4, 32, 1, 7), (64, 1.0, 4, 2, 0.05, 9, 1, 1)])
def test_pipeline_schedule_is_topological_and_drains(L, N, T, Ns, K, dt, M, split, group):
    jobs = binding.pipeline_schedule(N, T, Ns, K, dt, M, split=split, group=group)
    gs = group if group > 0 else max(1, 8 * (64 // (8 if N <= 64 else 16 if N <= 128 else 32 if N <= 256 else 64)) // 3)
    groups = (M - 1 + gs - 1) // gs
    is_split = (groups >= 2) if split < 0 else bool(split)
    steps = max(1, math.ceil(T / Ns / dt - 1e-9))
    # fine slices F(k, n) for n > k; slices n <= k of level k >= 1 are copies
    want = {(1, k, n, 0) for k in range(K) for n in range(k + 1, Ns + 1)}
    want |= {(4, k, n, 0) for k in range(1, K + 1) for n in range(1, min(k, Ns) + 1)}
    real = [(k, n) for k in range(K + 1) for n in range(1, Ns + 1) if not (k >= 1 and n <= k)]
    if is_split:
        want |= {(t, k, n, x) for t in (2, 3) for (k, n) in real for x in range(groups)}
    else:
        want |= {(0, k, n, 0) for (k, n) in real}
    assert len(jobs) == len(want) and set(jobs) == want
    pos = {j: i for i, j in enumerate(jobs)}
    for j in jobs:
        for d in _deps(j, K, groups, is_split):
            assert pos[d] < pos[j], (j, d)
    # ticket scheduling with W workers: each takes the next job and waits for
    # its dependencies (durations in nonlinear evaluations)
    dur = {0: 2 * (M - 1), 1: 4 * steps, 2: gs, 3: gs, 4: 0.1}
    for W in (1, 3, 256):
        free = [0.0] * W
        end = {}
        for j in jobs:
            w = min(range(W), key=lambda i: free[i])
            start = max([free[w]] + [end[d] for d in _deps(j, K, groups, is_split)])
            end[j] = start + dur[j[0]]
            free[w] = end[j]
        assert max(end.values()) <= sum(dur[j[0]] for j in jobs) + 1e-9


def test_batch_and_options_reject_bad_arguments(L):
    assert L.aparareal_solve_batch(None, 1, None) == -1
    assert L.aparareal_solve_batch(None, -1, None) == -1
    assert L.aparareal_solve_batch(None, 0, None) == 0
    items = (binding.BatchItem * 1)()
    assert L.aparareal_solve_batch(items, 1, None) == -1           # null context
    assert b"null context" in L.aparareal_last_error()
    assert L.aparareal_set_option(None, binding.AP_OPT_SPLIT, 1) == -1
    v = ctypes.c_int(0)
    assert L.aparareal_get_option(None, binding.AP_OPT_GROUP, ctypes.byref(v)) == -1


def test_batch_item_layout_matches_header():
    names = [f[0] for f in binding.BatchItem._fields_]
    assert names == ["ctx", "u0", "params", "U_out", "resid"]
    assert ctypes.sizeof(binding.BatchItem) == 8 + 8 + 56 + 8 + 8


def test_serving_rejects_bad_arguments(L):
    assert not L.aparareal_serve_create(0, 4)
    assert not L.aparareal_serve_create(1 << 30, 0)
    t = ctypes.c_ulonglong(0)
    p = binding.SolveParams(1.0, 4, 2, 0.01, 8, 0.0, 0.0, 0)
    assert L.aparareal_serve_submit(None, 64, 0.1, 1.0, 0.0, None, ctypes.byref(p), ctypes.byref(t)) == -1
    assert L.aparareal_serve_poll(None, 1, None, None, None) == -1
    assert L.aparareal_serve_destroy(None) == -1
    assert b"null server" in L.aparareal_last_error()


@pytest.mark.parametrize("Ns,K", [(64, 8), (16, 5), (3, 9), (256, 10)])
def test_counted_work_matches_the_jobs_run(L, Ns, K):
    # the benchmark counts fine slices and coarse steps actually computed
    from paper_1303_6615_amd import metrics
    jobs = binding.pipeline_schedule(256, 1.0, Ns, K, 0.001, 32, split=0)
    fine = sum(1 for j in jobs if j[0] == 1)
    coarse = sum(1 for j in jobs if j[0] == 0)
    gp, flops = metrics.pipelined_work(256, Ns, K, 7, 32)
    assert gp == fine * 7 * 256
    assert flops == pytest.approx(metrics.fine_flops(256, fine, 7) + coarse * metrics.coarse_step_flops(256, 32))
