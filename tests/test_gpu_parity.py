"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over all 3*N grid values, worst state):
  * FP64 mode: 1e-11 for propagators and the full solve, 5e-13 for single N
    (a few ulps times log2 N, amplified by the i*k derivative at high k);
  * FP32 mode: 2e-5 for propagators and the solve; single N at 1e-5 in the
    H^-1 norm (mode-k errors divided by 1 + k): N differentiates quadratic
    products once, and FP32 rounding of the products is white in k, so its
    image under i*k grows with k; H^-1 measures the products' rounding itself.
    In the plain relative L2 norm single N is held to 1e-7 x Kd.
"""
import numpy as np
import pytest

import oracle as O
from paper_1303_6615_amd.inputs import C1, C2, SolveConfig, seeded_state, NU_BY_NX

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
    if prec == FP32:
        # plain relative L2: the FP32 rounding of the products is white over
        # the retained band and N differentiates it once, so the error of mode
        # k grows with k while N's energy sits at low k; the relative error
        # grows with Kd = N/3, measured 4-5.4e-8 x Kd for N = 64..2048
        assert _rel(got, ref) < 1e-7 * (n // 3)


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
    (512, 0.01, 1.0 / 64, 32, FP32, 2e-5),
    (512, 0.1, 0.05, 10, FP64, 1e-11),
    (2048, 0.01, 0.01, 20, FP32, 2e-5),
    (2048, 0.001, 0.002, 20, FP64, 1e-11),
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


@pytest.mark.parametrize("n,prec,strang", [(64, FP64, False), (128, FP32, False), (256, FP32, False),
                                            (256, FP32, True), (512, FP64, False)])
def test_fine_batch_slices_stepped_together_equal_alone(torch_cuda, n, prec, strang):
    # a workgroup steps several slices at once (16, 10, 5, 2 for N = 64 .. 512);
    # each rounds exactly as alone, whatever the batch and its ragged last group
    torch = torch_cuda
    nu = NU_BY_NX[n]
    u = torch.tensor(_states(n, 13, 11 * n), device="cuda")
    with _ctx(n, 0.01, nu) as ctx:
        run = (lambda x: ctx.strang_batch(x, 0.01, 3, precision=prec)) if strang else \
              (lambda x: ctx.fine_batch(x, 0.01, 3, precision=prec))
        together = run(u)
        alone = torch.cat([run(u[i:i + 1]) for i in range(u.shape[0])])
    assert torch.equal(together, alone)


_G512 = SolveConfig("grouped-n512", nx=512, eps=0.01, nu=NU_BY_NX[512], T=0.2, slices=14, K=3, dt=0.01 / 20,
                    Mbar=16, k_ic=64, seed=31)
_G1024 = SolveConfig("grouped-n1024", nx=1024, eps=0.01, nu=NU_BY_NX[1024], T=0.1, slices=9, K=3, dt=0.01 / 20,
                     Mbar=16, k_ic=128, seed=32)


@pytest.mark.parametrize("cfg,prec,fine_kind", [(C1, FP64, 0), (C2, FP32, 0), (C2, FP32, 1), (_G512, FP32, 0),
                                                (_G1024, FP32, 0), (_G1024, FP32, 1), (_G512, FP64, 0)])
def test_grouped_fine_jobs_change_no_value(torch_cuda, cfg, prec, fine_kind):
    # fine jobs of the pipelined solve over up to 16 / 5 consecutive slices
    # (AP_OPT_FINE_GROUP) give the single-slice results bitwise; at N = 512
    # and 1024 the FP32 ETDRK4 jobs hold two (slice, mode) items per thread
    # (5 slices in two rounds of transforms, 2 slices)
    from paper_1303_6615_amd.binding import AP_OPT_FINE, AP_OPT_FINE_GROUP
    torch = torch_cuda
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_FINE, fine_kind)
        ctx.set_option(AP_OPT_FINE_GROUP, 1)
        U1, r1 = _solve(ctx, torch, cfg, prec)
        U1, r1 = U1.clone(), r1.clone()
        for fg in (3, 64):
            ctx.set_option(AP_OPT_FINE_GROUP, fg)
            Ug, rg = _solve(ctx, torch, cfg, prec)
            assert torch.equal(U1, Ug) and torch.equal(r1, rg), fg


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
    (512, 0.01, 1.0 / 64, 32, FP32, 2e-5),
    (512, 0.001, 1.0 / 128, 32, FP64, 1e-12),
    (2048, 0.01, 1.0 / 32, 32, FP32, 2e-5),
    (2048, 0.1, 0.125, 16, FP64, 1e-12),
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
    # AP_OPT_SWEEPS with tol > 0 runs the iteration-by-iteration sweeps (tol far
    # below reach: all K iterations); otherwise the pipelined persistent launch
    # with slice skipping.  Same values.
    from paper_1303_6615_amd.binding import AP_OPT_SWEEPS
    torch = torch_cuda
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        Up, rp = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=prec)
        ctx.set_option(AP_OPT_SWEEPS, 1)
        Us, rs = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, tol=1e-300, precision=prec)
        ctx.set_option(AP_OPT_SWEEPS, 0)
        Up2, rp2 = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(Up, Us) and torch.equal(rp, rs)
        assert torch.equal(Up, Up2) and torch.equal(rp, rp2)      # run to run


@pytest.mark.parametrize("cfg,prec,tol", [(C1, FP64, 1e-6), (C2, FP32, 1e-5)])
def test_tolerance_stops_early(torch_cuda, cfg, prec, tol):
    # the pipelined launch decides on the device to stop after the first
    # iteration with r^k <= tol; the host-checked sweeps give the same values,
    # and the output equals a solve run for exactly that many iterations
    from paper_1303_6615_amd.binding import AP_OPT_SWEEPS
    torch = torch_cuda
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        U, r = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, tol=tol, precision=prec)
        ctx.set_option(AP_OPT_SWEEPS, 1)
        Us, rs = ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, tol=tol, precision=prec)
        ctx.set_option(AP_OPT_SWEEPS, 0)
        torch.cuda.synchronize()
        assert torch.equal(U, Us) and torch.equal(r, rs)
        r = r.cpu().numpy()
        ran = r[r >= 0]
        assert 0 < ran.size < cfg.K and ran[-1] <= tol and np.all(ran[:-1] > tol)
        assert np.all(r[ran.size:] == -1.0)
        Uk, rk = ctx.solve(u0, cfg.T, cfg.slices, ran.size, cfg.dt, cfg.Mbar, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(U, Uk) and np.array_equal(rk.cpu().numpy(), ran)


@pytest.mark.parametrize("cfg,prec,split", [(C1, FP64, 0), (C1, FP64, 1), (C2, FP32, 1)])
def test_slice_skipping_changes_no_value(torch_cuda, cfg, prec, split):
    # slices n <= k are exact after k iterations: copying them instead of
    # recomputing them leaves every value unchanged
    from paper_1303_6615_amd.binding import AP_OPT_SKIP, AP_OPT_SPLIT
    torch = torch_cuda
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_SPLIT, split)
        ctx.set_option(AP_OPT_SKIP, 0)
        Ua, ra = _solve(ctx, torch, cfg, prec)
        ctx.set_option(AP_OPT_SKIP, 1)
        Ub, rb = _solve(ctx, torch, cfg, prec)
    assert torch.equal(Ua, Ub) and torch.equal(ra, rb)


def _solve(ctx, torch, cfg, prec, **kw):
    U, r = ctx.solve(torch.tensor(cfg.initial_state(), device="cuda"), cfg.T, cfg.slices, cfg.K, cfg.dt,
                     cfg.Mbar, precision=prec, **kw)
    torch.cuda.synchronize()
    return U, r


@pytest.mark.parametrize("cfg,prec", [(C1, FP64), (C2, FP32)])
def test_split_coarse_steps_equal_single_workgroup_steps_bitwise(torch_cuda, cfg, prec):
    # A coarse step split over one workgroup per sample group sums the groups
    # in the same order as one workgroup does: identical bits, for the default
    # and an uneven group size.
    from paper_1303_6615_amd.binding import AP_OPT_SPLIT, AP_OPT_GROUP
    torch = torch_cuda
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        for group in (0, 3):
            ctx.set_option(AP_OPT_GROUP, group)
            ctx.set_option(AP_OPT_SPLIT, 1)
            Us, rs = _solve(ctx, torch, cfg, prec)
            ctx.set_option(AP_OPT_SPLIT, 0)
            Uw, rw = _solve(ctx, torch, cfg, prec)
            Uq, rq = _solve(ctx, torch, cfg, prec, tol=1e-300)
            assert torch.equal(Us, Uw) and torch.equal(rs, rw), group
            assert torch.equal(Us, Uq) and torch.equal(rs, rq), group


@pytest.mark.parametrize("fg", [1, 2])
def test_split_steps_with_short_fine_jobs(torch_cuda, fg):
    # eps = 0.1 with 16 slices of T = 0.1: two fine steps per slice, so fine
    # jobs end long before the coarse step they feed, and consumers are
    # already polling when a split step's finisher publishes.  Split and whole
    # coarse steps give the same bits, run after run, and the oracle's values.
    from paper_1303_6615_amd.binding import AP_OPT_FINE_GROUP, AP_OPT_SPLIT
    from paper_1303_6615_amd.inputs import SolveConfig
    torch = torch_cuda
    cfg = SolveConfig("short-fine-n512", nx=512, eps=0.1, nu=NU_BY_NX[512], T=0.1, slices=16, K=8, dt=0.1 / 20,
                      Mbar=32, k_ic=64, seed=21)
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_FINE_GROUP, fg)
        ctx.set_option(AP_OPT_SPLIT, 0)
        Uw, rw = _solve(ctx, torch, cfg, FP32)
        ctx.set_option(AP_OPT_SPLIT, 1)
        for rep in range(3):
            Us, rs = _solve(ctx, torch, cfg, FP32)
            assert torch.equal(Us, Uw) and torch.equal(rs, rw), rep
    Uref, rref = _oracle_solve(cfg)
    assert _rel(Uw.cpu().numpy(), Uref) < 2e-5
    assert np.all(np.abs(rw.cpu().numpy() - rref) <= 1e-3 * rref + 1e-6)


@pytest.mark.parametrize("split", [0, 1])
def test_tolerance_stop_matches_the_oracle(torch_cuda, split):
    # Alg. 4's while loop: the device-side stop after the first iteration
    # with r^k <= tol gives the oracle's tolerance-stopped iterate and
    # residuals (FP64; tol placed between two of the oracle's residuals)
    from paper_1303_6615_amd.binding import AP_OPT_SPLIT
    torch = torch_cuda
    cfg = C1
    _, rfull = _oracle_solve(cfg)
    stop = 3
    tol = float(np.sqrt(rfull[stop - 1] * rfull[stop - 2]))
    Uref, rref, _ = O.parareal_solve(cfg.initial_state(), cfg.nx, cfg.eps, cfg.F, cfg.nu, cfg.T, cfg.slices,
                                     cfg.K, cfg.fine_steps, cfg.Mbar, cfg.window, tol=tol)
    assert len(rref) == stop
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_SPLIT, split)
        U, r = _solve(ctx, torch, cfg, FP64, tol=tol)
    r = r.cpu().numpy()
    assert np.all(r[stop:] == -1.0) and np.all(r[:stop] >= 0)
    assert np.all(np.abs(r[:stop] - np.array(rref)) <= 1e-6 * np.array(rref) + 1e-12)
    assert _rel(U.cpu().numpy(), Uref) < 1e-11


def test_group_size_changes_rounding_only(torch_cuda):
    from paper_1303_6615_amd.binding import AP_OPT_GROUP
    torch = torch_cuda
    cfg = C1
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_GROUP, 1)
        U1, _ = _solve(ctx, torch, cfg, FP64)
        ctx.set_option(AP_OPT_GROUP, 0)
        U0, _ = _solve(ctx, torch, cfg, FP64)
    assert _rel(U1.cpu().numpy(), U0.cpu().numpy()) < 1e-13


# uneven problems of one batch: (N, eps, slices, K, T, M, seed); nu by grid size
_BATCH = [(128, 0.1, 8, 3, 0.4, 16, 11), (256, 0.01, 16, 4, 0.2, 32, 12), (512, 0.01, 6, 2, 0.06, 16, 13),
          (256, 0.001, 5, 5, 0.02, 8, 14)]


def _batch_problem(n, eps, S, K, T, M, seed):
    nu = NU_BY_NX[n]
    u0 = seeded_state(n, n // 8, seed)
    return dict(n=n, eps=eps, nu=nu, u0=u0, prm=dict(T=T, slices=S, K=K, dt_fine=eps / 20, M=M))


@pytest.mark.parametrize("prec,tol,which", [(FP32, 2e-5, [0, 1, 2, 3]), (FP32, 2e-5, [1, 3]),
                                            (FP64, 1e-11, [0, 1])])
def test_batch_of_uneven_problems(torch_cuda, prec, tol, which):
    # one persistent launch over problems of different N, eps, slices and K
    # (several grid sizes, or one); each problem's result equals its solve
    # alone bitwise, and the oracle within the precision's tolerance
    from paper_1303_6615_amd.binding import solve_batch
    torch = torch_cuda
    probs = [_batch_problem(*_BATCH[i]) for i in which]
    ctxs = [_ctx(q["n"], q["eps"], q["nu"]) for q in probs]
    try:
        items = [(c, torch.tensor(q["u0"], device="cuda"), q["prm"]) for c, q in zip(ctxs, probs)]
        got = solve_batch(items, precision=prec)
        torch.cuda.synchronize()
        for c, (_, u0, prm), (U, r), q in zip(ctxs, items, got, probs):
            Ua, ra = c.solve(u0, prm["T"], prm["slices"], prm["K"], prm["dt_fine"], prm["M"], precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(U, Ua) and torch.equal(r, ra), q["n"]
            steps = int(np.ceil(prm["T"] / prm["slices"] / prm["dt_fine"] - 1e-9))
            Uref, _, _ = O.parareal_solve(q["u0"], q["n"], q["eps"], 1.0, q["nu"], prm["T"], prm["slices"],
                                          prm["K"], steps, prm["M"], prm["T"] / prm["slices"] / q["eps"])
            assert _rel(U.cpu().numpy(), Uref) < tol, q["n"]
    finally:
        for c in ctxs:
            c.close()


def test_batch_of_more_problems_of_one_size_than_one_boundary_launch_takes(torch_cuda):
    # 70 problems at N = 64 and 2 at N = 128 in one batch: the boundary
    # transforms of a batch run one launch per grid size and per 64 problems,
    # so N = 64 takes two launches; every problem equals its solve alone
    # bitwise, and two of them the oracle
    from paper_1303_6615_amd.binding import solve_batch
    torch = torch_cuda
    probs = [_batch_problem(64, 0.1, 3 + i % 3, 2, 0.06, 8, 200 + i) for i in range(70)]
    probs += [_batch_problem(128, 0.1, 4, 2, 0.06, 8, 300 + i) for i in range(2)]
    ctxs = [_ctx(q["n"], q["eps"], q["nu"]) for q in probs]
    try:
        items = [(c, torch.tensor(q["u0"], device="cuda"), q["prm"]) for c, q in zip(ctxs, probs)]
        got = solve_batch(items, precision=FP32)
        torch.cuda.synchronize()
        for i, (c, (_, u0, prm), (U, r), q) in enumerate(zip(ctxs, items, got, probs)):
            Ua, ra = c.solve(u0, prm["T"], prm["slices"], prm["K"], prm["dt_fine"], prm["M"], precision=FP32)
            torch.cuda.synchronize()
            assert torch.equal(U, Ua) and torch.equal(r, ra), i
            if i in (0, 69):
                steps = int(np.ceil(prm["T"] / prm["slices"] / prm["dt_fine"] - 1e-9))
                Uref, _, _ = O.parareal_solve(q["u0"], q["n"], q["eps"], 1.0, q["nu"], prm["T"], prm["slices"],
                                              prm["K"], steps, prm["M"], prm["T"] / prm["slices"] / q["eps"])
                assert _rel(U.cpu().numpy(), Uref) < 2e-5, i
    finally:
        for c in ctxs:
            c.close()


def test_large_solve_first_slices_match_serial_oracle(torch_cuda):
    # The full 1024-point, 256-slice, K = 10 solve as the benchmark times it:
    # after K iterations the first K slices equal the serial fine solution
    # (parareal property), which the oracle computes slice by slice.
    from paper_1303_6615_amd.inputs import C3
    torch = torch_cuda
    cfg = C3
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        U, r = _solve(ctx, torch, cfg, FP32)
        U = U.cpu().numpy()
        U64, _ = _solve(ctx, torch, cfg, FP64)
        U64 = U64.cpu().numpy()
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(r.cpu().numpy()))
    u = O.project(O.to_spectral(cfg.initial_state()), cfg.nx)
    dT = cfg.T / cfg.slices
    for n in range(1, 4):
        u = O.fine_propagate(u, cfg.nx, cfg.eps, cfg.F, cfg.nu, dT, cfg.fine_steps)
        x = O.to_physical(u, cfg.nx)
        assert _rel(U[n], x) < 2e-5, n
        assert _rel(U64[n], x) < 1e-11, n
    # FP32 propagators with the FP64 correction against the all-FP64 run
    assert _rel(U, U64) < 2e-5


def test_autotune_picks_a_mapping_and_changes_rounding_only(torch_cuda):
    # The tuned mapping and job order leave values unchanged; the tuned group
    # size changes the summation order of the average only.  Later solves
    # equal solves of a fresh context with the options read back, and stay
    # within the FP32 budget of the oracle.
    from paper_1303_6615_amd.binding import AP_OPT_GROUP, AP_OPT_SPLIT, autotune
    torch = torch_cuda
    cfg = C2
    Uref, _ = _oracle_solve(cfg)
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        U0, _ = _solve(ctx, torch, cfg, FP32)
        U0 = U0.clone()
        u0 = torch.tensor(cfg.initial_state(), device="cuda")
        ms = autotune([(ctx, u0, dict(T=cfg.T, slices=cfg.slices, K=cfg.K, dt_fine=cfg.dt, M=cfg.Mbar))])
        split, group = ctx.get_option(AP_OPT_SPLIT), ctx.get_option(AP_OPT_GROUP)
        assert ms > 0 and split in (0, 1) and group >= 1
        U1, r1 = _solve(ctx, torch, cfg, FP32)
        with _ctx(cfg.nx, cfg.eps, cfg.nu) as fresh:
            fresh.set_option(AP_OPT_SPLIT, split)
            fresh.set_option(AP_OPT_GROUP, group)
            U2, r2 = _solve(fresh, torch, cfg, FP32)
        assert torch.equal(U1, U2) and torch.equal(r1, r2)
        assert _rel(U1.cpu().numpy(), U0.cpu().numpy()) < 1e-5
        assert _rel(U1.cpu().numpy(), Uref) < 2e-5


def _serve_all(srv, reqs, precision=FP32):
    import time
    tickets = [srv.submit(c.nx, c.eps, c.F, c.nu, c.initial_state(), c.T, c.slices, c.K, c.dt, c.Mbar,
                          precision=precision) for c in reqs]
    out = {}
    t_end = time.time() + 120
    while len(out) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.002)
    assert len(out) == len(tickets), "serving did not finish in time"
    return [out[t] for t in tickets]


def test_serving_results_equal_alone_solves(torch_cuda):
    # requests of uneven N, eps, T and slices through the serving loop: each
    # result equals the same solve run alone (continuous batching changes only
    # what runs beside a request), and within FP32 tolerance of the oracle
    from paper_1303_6615_amd.binding import Server
    from paper_1303_6615_amd.inputs import serving_requests
    torch = torch_cuda
    reqs = [c for c in serving_requests(40, seed=7, T_range=(0.05, 0.2)) if c.nx <= 512][:10]
    assert len(reqs) >= 6
    with Server(8 << 30, 8) as srv:
        got = _serve_all(srv, reqs)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["bytes_held"] == 0
    for c, (U, r, lat) in zip(reqs, got):
        assert lat > 0
        with _ctx(c.nx, c.eps, c.nu) as ctx:
            Ua, ra = _solve(ctx, torch, c, FP32)
        assert np.array_equal(U, Ua.cpu().numpy()) and np.array_equal(r, ra.cpu().numpy()), c.name
    c = reqs[0]
    Uref, _, _ = O.parareal_solve(c.initial_state(), c.nx, c.eps, c.F, c.nu, c.T, c.slices, c.K, c.fine_steps,
                                  c.Mbar, c.window)
    assert _rel(got[0][0], Uref) < 2e-5


def test_serving_admission_by_memory_budget(torch_cuda):
    # a budget that holds one request at a time still serves them all, in
    # order; a request larger than the budget is refused at submission
    from paper_1303_6615_amd.binding import APError, Server
    from paper_1303_6615_amd.inputs import serving_requests
    reqs = serving_requests(3, seed=8, nxs=(256,), T_range=(0.05, 0.1))
    with Server(6 << 20, 8) as srv:
        got = _serve_all(srv, reqs)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["peak_bytes"] <= 6 << 20
        big = serving_requests(1, seed=9, nxs=(2048,), T_range=(4.0, 4.0))[0]
        with pytest.raises(APError):
            srv.submit(big.nx, big.eps, big.F, big.nu, big.initial_state(), big.T, big.slices, big.K, big.dt,
                       big.Mbar)
    assert all(np.all(np.isfinite(U)) for U, _, _ in got)


def test_graph_replay_equals_eager_solves(torch_cuda):
    # the pipelined solve captured into a hipGraph and replayed: every replay,
    # with eager work and host synchronisation between replays, equals the
    # eagerly enqueued solve; a new input at the same address is picked up
    from paper_1303_6615_amd.binding import AP_OPT_GRAPH
    torch = torch_cuda
    cfg = C2
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    u1 = torch.tensor(seeded_state(cfg.nx, cfg.k_ic, 99), device="cuda")
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        def solve(u, out, resid):
            return ctx.solve(u, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=FP32, out=out, resid=resid)
        out = torch.empty((cfg.slices + 1, 3, cfg.nx), dtype=torch.float64, device="cuda")
        resid = torch.empty((cfg.K,), dtype=torch.float64, device="cuda")
        ref0 = [t.clone() for t in solve(u0, out, resid)]
        x = u0.clone()
        solve(u1.clone(), out, resid)
        ref1 = [t.clone() for t in (out, resid)]
        ctx.set_option(AP_OPT_GRAPH, 1)
        for rep in range(4):
            src = u0 if rep % 2 == 0 else u1
            x.copy_(src)
            junk = torch.randn(1 << 16, device="cuda").sum()          # eager work between replays
            solve(x, out, resid)
            torch.cuda.synchronize()
            want = ref0 if rep % 2 == 0 else ref1
            assert torch.equal(out, want[0]) and torch.equal(resid, want[1]), rep
            assert torch.isfinite(junk)


def test_batch_problems_stop_on_their_own_tolerance(torch_cuda):
    from paper_1303_6615_amd.binding import _batch_items, _check, _stream, lib
    torch = torch_cuda
    probs = [_batch_problem(*_BATCH[i]) for i in (0, 1, 3)]
    tols = [1e-4, 0.0, 1e-5]
    ctxs = [_ctx(q["n"], q["eps"], q["nu"]) for q in probs]
    try:
        items = [(c, torch.tensor(q["u0"], device="cuda"), q["prm"]) for c, q in zip(ctxs, probs)]
        arr, outs = _batch_items(items, FP32)
        for i, t in enumerate(tols):
            arr[i].params.tol = t
        _check(lib().aparareal_solve_batch(arr, len(items), _stream(torch)))
        torch.cuda.synchronize()
        stopped = 0
        for c, (_, u0, prm), (U, r, _), t in zip(ctxs, items, outs, tols):
            Ua, ra = c.solve(u0, prm["T"], prm["slices"], prm["K"], prm["dt_fine"], prm["M"], tol=t, precision=FP32)
            torch.cuda.synchronize()
            assert torch.equal(U, Ua) and torch.equal(r, ra)
            stopped += int((r.cpu().numpy() < 0).any())
        assert stopped >= 1
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("n,eps,dT,steps,prec,tol", [(64, 0.01, 0.0625, 125, FP64, 1e-11), (256, 0.01, 0.03125, 63, FP32, 2e-5),
                                                     (1024, 0.001, 0.004, 40, FP32, 2e-5), (512, 0.1, 0.05, 1, FP64, 1e-11)])
def test_strang_batch(torch_cuda, n, eps, dT, steps, prec, tol):
    from oracle.strang import strang_propagate
    torch = torch_cuda
    nu = NU_BY_NX[n]
    u = _states(n, 3, 300 + n)
    ref = O.to_physical(strang_propagate(O.project(O.to_spectral(u), n), n, eps, 1.0, nu, dT, steps), n)
    with _ctx(n, eps, nu) as ctx:
        got = ctx.strang_batch(torch.tensor(u, device="cuda"), dT, steps, precision=prec).cpu().numpy()
    assert _rel(got, ref) < tol


@pytest.mark.parametrize("cfg,prec,tol,fine_kind,coarse_kind", [(C1, FP64, 1e-11, 1, 1), (C2, FP32, 2e-5, 1, 1),
                                                                (C1, FP64, 1e-11, 1, 0), (C2, FP32, 2e-5, 0, 1)])
def test_strang_and_standard_parareal_solves(torch_cuda, cfg, prec, tol, fine_kind, coarse_kind):
    # Strang fine slices (Alg. 3) and/or the one-step Strang coarse solver of
    # standard parareal, through the pipelined launch, against the oracle
    from oracle.strang import strang_propagate
    from paper_1303_6615_amd.binding import AP_OPT_COARSE, AP_OPT_FINE
    torch = torch_cuda
    dT = cfg.T / cfg.slices
    coarse = (lambda v: strang_propagate(v, cfg.nx, cfg.eps, cfg.F, cfg.nu, dT, 1)) if coarse_kind else None
    fine = (lambda v: strang_propagate(v, cfg.nx, cfg.eps, cfg.F, cfg.nu, dT, cfg.fine_steps)) if fine_kind else None
    Uref, rref, _ = O.parareal_solve(cfg.initial_state(), cfg.nx, cfg.eps, cfg.F, cfg.nu, cfg.T, cfg.slices, cfg.K,
                                     cfg.fine_steps, cfg.Mbar, cfg.window, coarse=coarse, fine=fine)
    with _ctx(cfg.nx, cfg.eps, cfg.nu) as ctx:
        ctx.set_option(AP_OPT_FINE, fine_kind)
        ctx.set_option(AP_OPT_COARSE, coarse_kind)
        U, r = _solve(ctx, torch, cfg, prec)
    assert _rel(U.cpu().numpy(), Uref) < tol
    floor = 1e-13 if prec == FP64 else 1e-6
    assert np.all(np.abs(r.cpu().numpy() - np.array(rref)) <= 1e-3 * np.array(rref) + floor)


def test_paper_experiment_replay_converges(torch_cuda):
    # the paper's eps = 1 experiment (analytic height, mu = 1e-4, dT = 3/10,
    # dt = 1/200, 60 slices): the error against the serial fine solution falls
    # with every iteration for asymptotic and standard parareal
    from paper_1303_6615_amd.replay import run_case
    out = run_case(1.0, torch=torch_cuda)
    for method in ("asymptotic", "standard"):
        e = out[method]["error_by_k"]
        assert all(e[k + 1] < e[k] for k in range(len(e) - 1)), (method, e)
        assert e[-1] < 1e-3, (method, e)
        assert out[method]["tau_f_us"] > 0 and out[method]["measured_speedup_k5"] > 1


def test_replay_asymptotic_configuration_matches_the_oracle(torch_cuda):
    # the replay's eps = 1e-1 asymptotic parareal (Sec. 6.2 parameters as the
    # replay reads them: analytic height, N = 128, mu = 1e-4, dT = 3 eps,
    # Strang fine steps of eps/25 (Alg. 3), 150 slices, Mbar = 10, slow window
    # 5 eps, K = 5) through the pipelined launch, FP64, against the oracle's
    # Alg. 4 with the same fine and coarse solvers (Alg. 2 coarse step)
    from oracle.strang import strang_propagate
    from paper_1303_6615_amd.binding import AP_OPT_COARSE, AP_OPT_FINE
    from paper_1303_6615_amd.inputs import paper_height_state
    from paper_1303_6615_amd.replay import CASES, K_MAX, NU, NX
    torch = torch_cuda
    eps = 0.1
    c = CASES[eps]
    T, S, dT = c["slices"] * c["adT"], c["slices"], c["adT"]
    steps = int(np.ceil(dT / c["adt"] - 1e-9))
    T0 = c["window"] / eps
    u0 = paper_height_state(NX)
    Uref, rref, _ = O.parareal_solve(u0, NX, eps, 1.0, NU, T, S, K_MAX, steps, c["Mbar"], T0,
                                     fine=lambda v: strang_propagate(v, NX, eps, 1.0, NU, dT, steps))
    with _ctx(NX, eps, NU) as ctx:
        ctx.set_option(AP_OPT_FINE, 1)
        ctx.set_option(AP_OPT_COARSE, 0)
        U, r = ctx.solve(torch.tensor(u0, device="cuda"), T, S, K_MAX, c["adt"], c["Mbar"], T0=T0, precision=FP64)
        torch.cuda.synchronize()
    U, r = U.cpu().numpy(), r.cpu().numpy()
    assert _rel(U, Uref) < 1e-11
    assert np.all(np.abs(r - np.array(rref)) <= 1e-6 * np.array(rref) + 1e-13), (r, rref)


@pytest.mark.parametrize("n,eps,dT,steps,prec,tol", [
    (256, 0.01, 0.03125, 8, FP32, 2e-5), (1024, 0.001, 1.0 / 256, 6, FP32, 2e-5),
    (512, 0.01, 1.0 / 64, 5, FP64, 1e-11), (1024, 0.01, 1.0 / 64, 4, FP64, 1e-11),
    (64, 0.01, 1.0 / 16, 9, FP64, 1e-11), (2048, 0.01, 0.01, 3, FP64, 1e-11)])
def test_fine_batch_configurations_and_their_autotuner(torch_cuda, tmp_path, monkeypatch, n, eps, dT, steps, prec,
                                                       tol):
    # every compiled configuration of the fine batch (workgroup shape c % 3,
    # FFT plan c // 3, plan 1 from N = 256 on) keeps the oracle's values; the
    # workgroup shape gives the same bits (a slice rounds the same way whatever
    # workgroup steps it), and so does plan 1 except at N = 1024, whose plan 1
    # has other radices; the autotuner keeps the fastest configuration,
    # records it in the tuning cache, and a new context reads it back
    from paper_1303_6615_amd.binding import AP_OPT_FINE_SHAPE, AP_FINE_CONFIGS, APError
    torch = torch_cuda
    monkeypatch.setenv("APARAREAL_TUNE_CACHE", str(tmp_path / "tune.txt"))
    nu = NU_BY_NX[n]
    u = _states(n, 37, 17 * n)
    ud = torch.tensor(u, device="cuda")
    uh = O.project(O.to_spectral(u[:4]), n)
    ref = O.to_physical(O.fine_propagate(uh, n, eps, 1.0, nu, dT, steps), n)
    configs = list(range(AP_FINE_CONFIGS if n >= 256 else 3))
    with _ctx(n, eps, nu) as ctx:
        outs, shapes = {}, {}
        for c in configs:
            ctx.set_option(AP_OPT_FINE_SHAPE, c)
            outs[c] = ctx.fine_batch(ud, dT, steps, precision=prec)
            shapes[c] = ctx.fine_shape(prec)
        torch.cuda.synchronize()
        if n < 256:
            with pytest.raises(APError):
                ctx.set_option(AP_OPT_FINE_SHAPE, 3)
        assert len({shapes[c][1] for c in range(3)}) == 3, shapes       # three distinct workgroup sizes
        for c in configs:
            assert shapes[c][0] == c
            same = c < 3 or n != 1024
            if same:
                assert torch.equal(outs[c], outs[0]), c
            else:
                assert torch.equal(outs[c], outs[3]), c                 # shapes of plan 1 agree bitwise
            assert _rel(outs[c][:4].cpu().numpy(), ref) < tol, c
        ctx.set_option(AP_OPT_FINE_SHAPE, -1)
        best, ms = ctx.autotune_fine(ud, dT, steps, precision=prec)
        assert best in configs and all(ms[c] > 0 for c in configs) and ms[best] == min(ms[c] for c in configs)
        assert all(ms[c] == -1 for c in range(AP_FINE_CONFIGS) if c not in configs)
        assert ctx.fine_shape(prec)[0] == best
        assert torch.equal(ctx.fine_batch(ud, dT, steps, precision=prec), outs[best])
    with _ctx(n, eps, nu) as fresh:
        assert fresh.fine_shape(prec)[0] == best
    assert f" {n} {prec} {best}" in (tmp_path / "tune.txt").read_text()
