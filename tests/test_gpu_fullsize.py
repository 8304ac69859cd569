"""Full-size parity: the HIP path at the workload sizes, in the launch
configuration the benchmark times (schedule autotuned), against stored FP64
oracle results.

The stored results (tests/golden/solve_*.npz, tests/golden/mixed64.npz) are
written by tests/golden/make_golden.py, which calls only the oracle on the
seeded inputs; at these sizes the oracle needs minutes to an hour of CPU time,
too long to run inside a test.  Per-slice tolerance on the final iterate U^K
(relative L2 over the 3 N grid values of each slice): 2e-5 with FP32
propagators and the FP64 correction, 1e-11 all in FP64.  Residual histories
follow the oracle's: in FP64 to 1e-6 relative; in FP32 to 1e-3 relative above
a floor of 1e-7 per slice.  The FP32 propagators round: each fine or coarse
step differs from its FP64 value by a few 1e-8 relative, the correction
carries those differences along the slices, and once two iterates differ by
less than an FP32 ulp, G_new - G_old is zero or one ulp.  So the FP32
residual levels off at 1e-8 to 3e-8 x Ns where the FP64 one keeps falling
(measured: 1.4-3e-6 at 256 slices; 8e-6 against the oracle's 3e-6 at the
first iteration of a 211-slice problem whose iterations converge at once).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1303_6615_amd.inputs import C1, C2, C3, mixed_batch

pytestmark = pytest.mark.gpu

FP32, FP64 = 0, 1
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _physical(Uk, nx):
    """Retained-mode spectral states [..., 3, Kd+1] -> grid values [..., 3, N]."""
    full = np.zeros(Uk.shape[:-1] + (nx // 2 + 1,), dtype=np.complex128)
    full[..., :Uk.shape[-1]] = Uk
    return O.to_physical(full, nx)


def _rel_per_slice(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _resid_ok(r, rref, prec, slices):
    if prec == FP64:
        return np.all(np.abs(r - rref) <= 1e-6 * rref + 1e-13)
    return np.all(np.abs(r - rref) <= 1e-3 * rref + 1e-7 * slices)


def _golden(cfg):
    path = os.path.join(GOLDEN, f"solve_{cfg.name}.npz")
    with np.load(path) as z:
        return _physical(z["U"], cfg.nx), z["r"]


def _tuned_solve(torch, cfg, prec):
    from paper_1303_6615_amd.binding import Context, autotune
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    with Context(cfg.nx, cfg.eps, cfg.F, cfg.nu) as ctx:
        autotune([(ctx, u0, dict(T=cfg.T, slices=cfg.slices, K=cfg.K, dt_fine=cfg.dt, M=cfg.Mbar))],
                 precision=prec)
        U, r = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=prec)
        torch.cuda.synchronize()
        return U.cpu().numpy(), r.cpu().numpy()


@pytest.mark.parametrize("cfg,prec,tol", [
    (C1, FP64, 1e-11),
    (C2, FP32, 2e-5), (C2, FP64, 1e-11),
    (C3, FP32, 2e-5), (C3, FP64, 1e-11),
])
def test_every_slice_of_the_solve_matches_the_oracle(torch_cuda, cfg, prec, tol):
    # eq. HMM parareal iteration (Alg. 4): all Ns + 1 slices of U^K
    Uref, rref = _golden(cfg)
    print(f"[fullsize] {cfg.name} prec={prec}", flush=True)
    U, r = _tuned_solve(torch_cuda, cfg, prec)
    assert U.shape == Uref.shape and np.all(np.isfinite(U))
    err = _rel_per_slice(U, Uref)
    print(f"[fullsize] worst slice rel L2 {err.max():.3e}", flush=True)
    assert np.all(err <= tol), (int(np.argmax(err)), float(err.max()))
    assert _resid_ok(r, rref, prec, cfg.slices), (r, rref)


def test_every_problem_of_the_mixed_batch_matches_the_oracle(torch_cuda):
    # the 64 uneven problems in one persistent launch, autotuned as the
    # benchmark runs them; per problem, sampled slices of U^K and the residuals
    from paper_1303_6615_amd.binding import Context, _batch_items, _check, _stream, autotune, lib
    torch = torch_cuda
    probs = mixed_batch(64)
    print("[fullsize] mixed batch of 64", flush=True)
    ctxs = [Context(c.nx, c.eps, c.F, c.nu) for c in probs]
    try:
        items = [(x, torch.tensor(c.initial_state(), device="cuda"),
                  dict(T=c.T, slices=c.slices, K=c.K, dt_fine=c.dt, M=c.Mbar)) for x, c in zip(ctxs, probs)]
        autotune(items, precision=FP32)
        arr, outs = _batch_items(items, FP32)
        _check(lib().aparareal_solve_batch(arr, len(items), _stream(torch)))
        torch.cuda.synchronize()
        got = [(U.cpu().numpy(), r.cpu().numpy()) for U, r, _ in outs]
    finally:
        for x in ctxs:
            x.close()
    worst, worst_r = 0.0, 0.0
    with np.load(os.path.join(GOLDEN, "mixed64.npz")) as z:
        for i, (c, (U, r)) in enumerate(zip(probs, got)):
            sl = z[f"p{i}_slices"]
            Uref = _physical(z[f"p{i}_U"].astype(np.complex128), c.nx)
            rref = z[f"p{i}_r"]
            assert np.all(np.isfinite(U)), i
            err = _rel_per_slice(U[sl], Uref)
            worst = max(worst, float(err.max()))
            worst_r = max(worst_r, float(np.max(np.abs(r - rref) / c.slices)))
            assert np.all(err <= 2e-5), (i, c.nx, c.eps, c.slices, float(err.max()))
            assert _resid_ok(r, rref, FP32, c.slices), (i, r, rref)
    print(f"[fullsize] mixed batch worst rel L2 {worst:.3e}, worst residual difference per slice "
          f"{worst_r:.3e}", flush=True)
