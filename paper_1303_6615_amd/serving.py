"""Serving measurement: a Poisson stream of solve requests through the
library's serving loop (FP32 propagators, continuous batching), and the same
arrival trace through the plain per-request FP64 path (one solve at a time,
in arrival order, no batching).  Host-side driver only; every solve runs in
the library."""
from __future__ import annotations

import time

import numpy as np


def _percentiles(lat):
    lat = np.asarray(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def closed_loop_rate(srv, reqs, precision=0) -> float:
    """Solves/s with every request submitted at once (saturated server)."""
    t0 = time.perf_counter()
    tickets = [srv.submit(c.nx, c.eps, c.F, c.nu, c.initial_state(), c.T, c.slices, c.K, c.dt, c.Mbar,
                          precision=precision) for c in reqs]
    pending = dict(zip(tickets, reqs))
    while pending:
        for t in list(pending):
            try:
                done = srv.poll(t) is not None
            except Exception as e:
                c = pending[t]
                raise RuntimeError(f"request {c.name} (N={c.nx}, eps={c.eps}, T={c.T:.3f}, slices={c.slices}) "
                                   f"failed: {e}") from e
            if done:
                del pending[t]
        time.sleep(0.0005)
    return len(reqs) / (time.perf_counter() - t0)


def open_loop(srv, reqs, arrivals, precision=0, keep=()) -> dict:
    """Submit request i at arrivals[i] (s after start); returns solves/s over
    first arrival to last completion, submit-to-completion latencies, and the
    results (U, resid) of the requests whose indices are in `keep`."""
    states = [c.initial_state() for c in reqs]
    keep = set(keep)
    t0 = time.perf_counter()
    tickets, done, kept = [], {}, {}
    i = 0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while i < len(reqs) and arrivals[i] <= now:
            c = reqs[i]
            tickets.append(srv.submit(c.nx, c.eps, c.F, c.nu, states[i], c.T, c.slices, c.K, c.dt, c.Mbar,
                                      precision=precision))
            i += 1
        for j, t in enumerate(tickets):
            if t not in done:
                try:
                    r = srv.poll(t)
                except Exception:
                    done[t] = (None, time.perf_counter() - t0)      # failed request
                    continue
                if r is not None:
                    done[t] = (r[2], time.perf_counter() - t0)
                    if j in keep:
                        kept[j] = (r[0], r[1])
        time.sleep(0.0002)
    lat = [done[t][0] for t in tickets if done[t][0] is not None]
    failed = sum(1 for t in tickets if done[t][0] is None)
    last = max(v[1] for v in done.values())
    p50, p99 = _percentiles(lat)
    return {"solves_per_s": len(lat) / (last - arrivals[0]), "p50_s": p50, "p99_s": p99, "failed": failed}, kept


def fifo_fp64(reqs, arrivals=None) -> dict:
    """Plain per-request FP64 path: in arrival order, one solve at a time on
    its own context, waiting for each to finish.  arrivals None: every
    request is there at the start (closed loop, back to back)."""
    import torch

    from .binding import Context, AP_PREC_FP64
    if arrivals is None:
        arrivals = np.zeros(len(reqs))
    ctxs = {}
    t0 = time.perf_counter()
    lat, last = [], 0.0
    for c, a in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        key = (c.nx, c.eps, c.F, c.nu)
        if key not in ctxs:
            ctxs[key] = Context(c.nx, c.eps, c.F, c.nu)
        u0 = torch.tensor(c.initial_state(), device="cuda")
        ctxs[key].solve(u0, c.T, c.slices, c.K, c.dt, c.Mbar, precision=AP_PREC_FP64)
        torch.cuda.synchronize()
        end = time.perf_counter() - t0
        lat.append(end - max(a, 0.0))
        last = end
    for ctx in ctxs.values():
        ctx.close()
    p50, p99 = _percentiles(lat)
    return {"solves_per_s": len(reqs) / (last - arrivals[0]), "p50_s": p50, "p99_s": p99}


def alone_check(reqs, kept) -> dict:
    """Re-runs each kept request alone (its own context, same options as a
    fresh solve) and compares it with its served result: bitwise equality is
    expected (jobs of different problems share no data), the gate is the
    FP32 tolerance, relative L2 <= 2e-5 per slice."""
    import torch

    from .binding import Context
    worst, equal = 0.0, 0
    for j, (U, r) in sorted(kept.items()):
        c = reqs[j]
        with Context(c.nx, c.eps, c.F, c.nu) as ctx:
            Ua, ra = ctx.solve(torch.tensor(c.initial_state(), device="cuda"), c.T, c.slices, c.K, c.dt, c.Mbar)
            torch.cuda.synchronize()
            Ua, ra = Ua.cpu().numpy(), ra.cpu().numpy()
        equal += int(np.array_equal(U, Ua) and np.array_equal(r, ra))
        a = U.reshape(U.shape[0], -1)
        b = Ua.reshape(Ua.shape[0], -1)
        worst = max(worst, float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1))))
    return {"requests": len(kept), "bitwise_equal": equal, "max_rel_l2": worst, "tolerance": 2e-5,
            "ok": bool(worst <= 2e-5)}


def run(n_requests: int = 512, warmup: int = 8, load: float = 0.7, budget_gib: float = 64.0, slots: int = 64,
        seed: int = 5, n_closed: int = 256, n_alone: int = 8) -> dict:
    """The serving workload: requests drawn like the mixed batch (N 128-2048,
    eps 0.1-0.001, T 0.5-4).
      closed loop: n_closed requests submitted at once to the server (batched
        FP32), and the same requests back to back through the plain FP64 path;
      open loop: n_requests Poisson arrivals at `load` x the closed-loop
        batched rate through the server, and the same arrival trace through
        the plain FP64 path;
      n_alone requests of the open-loop stream (seeded sample) re-run alone
        and compared with their served results."""
    from .binding import Server
    from .inputs import poisson_arrivals, serving_requests
    reqs = serving_requests(warmup + n_closed + n_requests, seed=seed)
    warm, pre, main = reqs[:warmup], reqs[warmup:warmup + n_closed], reqs[warmup + n_closed:]
    keep = sorted(np.random.default_rng(seed + 77).choice(len(main), size=min(n_alone, len(main)),
                                                          replace=False).tolist())
    with Server(int(budget_gib * (1 << 30)), slots) as srv:
        closed_loop_rate(srv, warm)
        sat = closed_loop_rate(srv, pre)
        rate = load * sat
        arr = poisson_arrivals(len(main), rate, seed=seed + 50)
        arr = arr - arr[0]
        served, kept = open_loop(srv, main, arr, keep=keep)
        st = srv.stats()
    fifo_closed = fifo_fp64(pre)
    base = fifo_fp64(main, arr)
    return {"unit": "solves/s, latency s", "requests": len(main), "closed_loop_requests": len(pre),
            "arrival_rate_per_s": round(rate, 4),
            "closed_loop": {"batched_fp32_solves_per_s": round(sat, 4),
                            "fifo_fp64_solves_per_s": round(fifo_closed["solves_per_s"], 4)},
            "batched_fp32": {k: round(v, 5) for k, v in served.items()},
            "fifo_fp64": {k: round(v, 5) for k, v in base.items()},
            "alone_vs_served": alone_check(main, kept),
            "batched_launches": int(st["launches"]), "peak_bytes": int(st["peak_bytes"])}
