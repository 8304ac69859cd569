"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over all 3*N grid values, worst state):
  * FP64 mode: 1e-11 for propagators and the full solve, 5e-13 for single N
    (a few ulps times log2 N, amplified by the i*k derivative at high k);
  * FP32 mode: 2e-5 for propagators and the solve; single N at 1e-5 in the
    H^-1 norm (mode-k errors divided by 1 + k): N differentiates quadratic
    products once, and FP32 rounding of the products is white in k, so its
    image under i*k grows with k; H^-1 measures the products' rounding itself.
"""
import numpy as np
import pytest

import oracle as O
from paper_1303_6615_amd.inputs import C1, C2, seeded_state, NU_BY_NX

pytestmark = pytest.mark.gpu

FP32, FP64 = 0, 1


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _ctx(n, eps, nu, F=1.0):
    from paper_1303_6615_amd.binding import Context
    return Context(n, eps, F, nu)


def _rel(a, b):
    a = np.asarray(a).reshape(-1, 3 * a.shape[-1])
    b = np.asarray(b).reshape(-1, 3 * b.shape[-1])
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def _rel_hm1(a, b, n):
    """Relative H^-1 distance: spectral differences weighted by 1/(1+k)."""
    w = 1.0 / (1.0 + np.arange(n // 2 + 1))
    da = O.to_spectral(np.asarray(a)) * w
    db = O.to_spectral(np.asarray(b)) * w
    num = np.sqrt(np.sum(np.abs(da - db) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(db) ** 2, axis=(-2, -1)))
    return float(np.max(num / den))


def _states(n, count, seed, amp=0.1, k_ic=None):
    return np.stack([seeded_state(n, k_ic or n // 8, seed + i, amplitude=amp) for i in range(count)])


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048])
@pytest.mark.parametrize("prec,tol", [(FP64, 5e-13), (FP32, 1e-5)])
def test_nonlinear(torch_cuda, n, prec, tol):
    torch = torch_cuda
    u = _states(n, 3, 100 + n, amp=1.0, k_ic=n // 3)
    u[1] += 0.01 * np.sin(np.arange(n) * (2 * np.pi / n) * (n // 2 - 1))   # out-of-band: projected away
    ref = O.nonlinear_physical(u)
    with _ctx(n, 0.01, NU_BY_NX[n]) as ctx:
        got = ctx.nonlinear(torch.tensor(u, device="cuda"), precision=prec).cpu().numpy()
    err = _rel(got, ref) if prec == FP64 else _rel_hm1(got, ref, n)
    assert err < tol


def test_empty_batch_is_noop(torch_cuda):
    torch = torch_cuda
    with _ctx(64, 0.01, 1e-4) as ctx:
        x = torch.zeros((0, 3, 64), dtype=torch.float64, device="cuda")
        assert ctx.fine_batch(x, 0.01, 3).shape == (0, 3, 64)


@pytest.mark.parametrize("n,eps,dT,steps,prec,tol", [
    (64, 0.01, 1.0 / 16, 125, FP64, 1e-11),
    (128, 0.1, 0.05, 7, FP64, 1e-11),
    (256, 0.01, 0.03125, 63, FP32, 2e-5),
    (256, 0.01, 0.03125, 63, FP64, 1e-11),
    (1024, 0.001, 1.0 / 256, 40, FP32, 2e-5),
])
def test_fine_batch(torch_cuda, n, eps, dT, steps, prec, tol):
    torch = torch_cuda
    nu = NU_BY_NX[n]
    u = _states(n, 5, 7 * n)
    uh = O.project(O.to_spectral(u), n)
    ref = O.to_physical(O.fine_propagate(uh, n, eps, 1.0, nu, dT, steps), n)
    with _ctx(n, eps, nu) as ctx:
        got = ctx.fine_batch(torch.tensor(u, device="cuda"), dT, steps, precision=prec).cpu().numpy()
    assert _rel(got, ref) < tol


@pytest.mark.parametrize("n,T0,M,prec,tol", [
    (64, 6.25, 16, FP64, 1e-12),
    (256, 3.125, 32, FP64, 1e-12),
    (256, 3.125, 32, FP32, 1e-5),
    (1024, 3.90625, 64, FP32, 1e-5),
    (512, 1.7, 13, FP64, 1e-12),
])
def test_average(torch_cuda, n, T0, M, prec, tol):
    torch = torch_cuda
    u = _states(n, 3, 11 * n, amp=0.5)
    uh = O.project(O.to_spectral(u), n)
    ref = O.to_physical(O.averaged_nonlinear(uh, n, 1.0, T0, M), n)
    with _ctx(n, 0.01, NU_BY_NX[n]) as ctx:
        got = ctx.average(torch.tensor(u, device="cuda"), T0, M, precision=prec).cpu().numpy()
    assert _rel(got, ref) < tol


@pytest.mark.parametrize("n,eps,dT,M,prec,tol", [
    (64, 0.01, 1.0 / 16, 16, FP64, 1e-12),
    (256, 0.01, 0.03125, 32, FP32, 2e-5),
    (256, 0.1, 0.1, 9, FP64, 1e-12),
])
def test_coarse(torch_cuda, n, eps, dT, M, prec, tol):
    torch = torch_cuda
    nu = NU_BY_NX[n]
    u = _states(n, 4, 13 * n)
    uh = O.project(O.to_spectral(u), n)
    ref = O.to_physical(O.coarse_propagate(uh, n, eps, 1.0, nu, dT, dT / eps, M), n)
    with _ctx(n, eps, nu) as ctx:
        got = ctx.coarse(torch.tensor(u, device="cuda"), dT, M, 0.0, precision=prec).cpu().numpy()
    assert _rel(got, ref) < tol


def _oracle_solve(cfg):
    U, res, _ = O.parareal_solve(cfg.initial_state(), cfg.nx, cfg.eps, cfg.F, cfg.nu, cfg.T,
                                 cfg.slices, cfg.K, cfg.fine_steps, cfg.Mbar, cfg.window)
    return U, np.array(res)


@pytest.mark.parametrize("cfg,prec,tol", [(C1, FP64, 1e-11), (C2, FP32, 2e-5)])
def test_solve(torch_cuda, cfg, prec, tol):
    torch = torch_cuda
    Uref, rref = _oracle_solve(cfg)
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        U, r = ctx.solve(torch.tensor(cfg.initial_state(), device="cuda"), cfg.T, cfg.slices, cfg.K,
                         cfg.dt, cfg.Mbar, precision=prec)
        U = U.cpu().numpy()
        r = r.cpu().numpy()
    assert _rel(U, Uref) < tol
    # residual history follows the oracle's (FP32 plateaus near its rounding level)
    floor = 1e-13 if prec == FP64 else 1e-6
    assert np.all(np.abs(r - rref) <= 1e-3 * rref + floor), (r, rref)


@pytest.mark.parametrize("cfg,prec", [(C1, FP64), (C2, FP32)])
def test_pipelined_solve_equals_iteration_order_bitwise(torch_cuda, cfg, prec):
    # tol > 0 runs the iteration-by-iteration sweeps (tol far below reach: all K
    # iterations); tol <= 0 runs the pipelined persistent launch.  Same bits.
    torch = torch_cuda
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        Up, rp = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=prec)
        Us, rs = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, tol=1e-300, precision=prec)
        Up2, rp2 = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(Up, Us) and torch.equal(rp, rs)
        assert torch.equal(Up, Up2) and torch.equal(rp, rp2)      # run to run


def test_tolerance_stops_early(torch_cuda):
    torch = torch_cuda
    cfg = C1
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        U, r = ctx.solve(torch.tensor(cfg.initial_state(), device="cuda"), cfg.T, cfg.slices, cfg.K,
                         cfg.dt, cfg.Mbar, tol=1e-6, precision=FP64)
        r = r.cpu().numpy()
    ran = r[r >= 0]
    assert 0 < ran.size < cfg.K and ran[-1] <= 1e-6 and np.all(ran[:-1] > 1e-6)
    assert np.all(r[ran.size:] == -1.0)
