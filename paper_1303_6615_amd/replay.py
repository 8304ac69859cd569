"""Replay of the paper's RSW experiments (Sec. 6.2) on the GPU path.

For eps = 1e-2, 1e-1 and 1, the analytic initial height of Sec. 6.2 (zero
velocities, max |h| = 1), mu = 1e-4, and the step sizes, windows and sample
counts the paper states, this runs
  * asymptotic parareal (Alg. 4: asymptotic coarse step, Strang fine steps of
    Alg. 3) and
  * standard parareal (Strang coarse step of length dT, Strang fine steps),
and reports, per iteration k = 0..5, the paper's error metric
max_n ||U_n^k - u(n dT)||_inf / ||u(n dT)||_inf against the serial fine
solution, together with the paper's estimated speedup (eq. speedup upper
bound) evaluated with job durations measured on the device, and the
measured wall time of the parareal solve against the serial fine chain on
the same GPU.

Readings (the paper states no grid, no final time and inconsistent windows):
  * grid N = 128;
  * T = slices x dT with 32 asymptotic slices at eps = 1e-2 (dT = 50 eps),
    150 at eps = 1e-1 (dT = 3 eps) and 60 at eps = 1 (dT = 3/10); standard
    parareal covers the same T with its own dT;
  * the window T0(eps) is read as slow time (150 eps, 5 eps, 3/10) and passed
    as the fast-time window T0 / eps;
  * "dT = eps = 1/20" at eps = 1e-1 is read as dT = eps.
"""
from __future__ import annotations

import time

import numpy as np

CASES = {
    # eps: asymptotic (dT, dt, slices, slow window, Mbar), standard (dT, dt)
    0.01: dict(adT=0.5, adt=0.01 / 25, slices=32, window=150 * 0.01, Mbar=450, sdT=4 * 0.01, sdt=0.01 / 25),
    0.1: dict(adT=0.3, adt=0.1 / 25, slices=150, window=5 * 0.1, Mbar=10, sdT=0.1, sdt=0.1 / 20),
    1.0: dict(adT=0.3, adt=1 / 200, slices=60, window=0.3, Mbar=10, sdT=0.3, sdt=1 / 200),
}
NX, NU, K_MAX = 128, 1e-4, 5


def _linf_err(U, ref):
    e = np.abs(U - ref).reshape(U.shape[0], -1).max(axis=1)
    r = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
    return float(np.max(e / r))


def _serial_fine(ctx, torch, u0, dT, steps, slices):
    """Serial Strang chain on the GPU (every slice boundary) and its wall time."""
    u = u0.clone().reshape(1, 3, NX)
    out = [u0.cpu().numpy()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, slices + 1):
        u = ctx.strang_batch(u, dT, steps, precision=1)
        out.append(u[0].cpu().numpy())
    torch.cuda.synchronize()
    return np.stack(out), time.perf_counter() - t0


def _method(ctx, torch, u0, T, slices, dT, dt, Mbar, T0, coarse_kind):
    from .binding import AP_OPT_COARSE, AP_OPT_FINE
    ctx.set_option(AP_OPT_FINE, 1)
    ctx.set_option(AP_OPT_COARSE, coarse_kind)
    errs, walls = [], []
    U_K = {}
    for K in range(K_MAX + 1):
        ctx.solve(u0, T, slices, K, dt, Mbar, T0=T0, precision=1)          # warm (tables, job list)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, _ = ctx.solve(u0, T, slices, K, dt, Mbar, T0=T0, precision=1)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        U_K[K] = U.cpu().numpy()
    # job durations of the K_MAX solve (device clock, 100 MHz)
    ctx.trace(True)
    ctx.solve(u0, T, slices, K_MAX, dt, Mbar, T0=T0, precision=1)
    torch.cuda.synchronize()
    tr = np.array(ctx.trace_read(), dtype=np.int64)
    ctx.trace(False)
    dur = (tr[:, 6] - tr[:, 5]) / 100.0 * 1e-6
    steps = max(1, int(np.ceil(T / slices / dt - 1e-9)))
    tau_f = float(np.median(dur[tr[:, 1] == 1])) / steps
    # coarse step latency: a whole job's duration, or for a split step the
    # span from its first stage-1 start to its last stage-2 end
    spans = {}
    for row in tr:
        if row[1] in (0, 2, 3):
            key = (int(row[2]), int(row[3]))
            lo, hi = spans.get(key, (row[5], row[6]))
            spans[key] = (min(lo, row[5]), max(hi, row[6]))
    tau_c = float(np.median([(hi - lo) / 100.0 * 1e-6 for lo, hi in spans.values()])) if spans else float("nan")
    return U_K, walls, tau_f, tau_c, steps


def run_case(eps: float, torch=None) -> dict:
    import torch as _torch

    from .binding import Context
    from .inputs import paper_height_state
    torch = torch or _torch
    c = CASES[eps]
    T = c["slices"] * c["adT"]
    u0 = torch.tensor(paper_height_state(NX), device="cuda")
    out = {"eps": eps, "N": NX, "nu": NU, "T": T}
    with Context(NX, eps, 1.0, NU) as ctx:
        # reference: the serial Strang chain with the asymptotic method's fine step
        a_steps = max(1, int(np.ceil(c["adT"] / c["adt"] - 1e-9)))
        ref, t_serial = _serial_fine(ctx, torch, u0, c["adT"], a_steps, c["slices"])
        U_K, walls, tau_f, tau_c, steps = _method(ctx, torch, u0, T, c["slices"], c["adT"], c["adt"], c["Mbar"],
                                                  c["window"] / eps, 0)
        errs = [_linf_err(U_K[k], ref) for k in range(K_MAX + 1)]
        N, M, nu_it = c["slices"], steps, K_MAX
        est = tau_f * N * M / (nu_it * (tau_f * M + tau_c * N + tau_c) + tau_c * N)
        out["asymptotic"] = {"dT": c["adT"], "dt": c["adt"], "slices": N, "M": M, "Mbar": c["Mbar"],
                             "T0_fast": c["window"] / eps, "error_by_k": errs,
                             "tau_f_us": tau_f * 1e6, "tau_c_us": tau_c * 1e6,
                             "estimated_speedup_k5": est, "wall_s_by_k": walls,
                             "serial_fine_wall_s": t_serial, "measured_speedup_k5": t_serial / walls[K_MAX]}
        # standard parareal over the same T: Strang coarse step of its own dT
        s_slices = int(round(T / c["sdT"]))
        s_steps = max(1, int(np.ceil(c["sdT"] / c["sdt"] - 1e-9)))
        sref, s_serial = _serial_fine(ctx, torch, u0, c["sdT"], s_steps, s_slices)
        U_S, s_walls, s_tau_f, s_tau_c, _ = _method(ctx, torch, u0, T, s_slices, c["sdT"], c["sdt"], 2, 0.0, 1)
        s_errs = [_linf_err(U_S[k], sref) for k in range(K_MAX + 1)]
        s_est = s_tau_f * s_slices * s_steps / (K_MAX * (s_tau_f * s_steps + s_tau_c * s_slices + s_tau_c)
                                                + s_tau_c * s_slices)
        out["standard"] = {"dT": c["sdT"], "dt": c["sdt"], "slices": s_slices, "M": s_steps, "error_by_k": s_errs,
                           "tau_f_us": s_tau_f * 1e6, "tau_c_us": s_tau_c * 1e6, "estimated_speedup_k5": s_est,
                           "wall_s_by_k": s_walls, "serial_fine_wall_s": s_serial,
                           "measured_speedup_k5": s_serial / s_walls[K_MAX]}
    return out


def main():
    import json
    for eps in (0.01, 0.1, 1.0):
        print(json.dumps(run_case(eps)), flush=True)


if __name__ == "__main__":
    main()
