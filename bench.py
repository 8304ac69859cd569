#!/usr/bin/env python3
"""Benchmark: asymptotic parareal solves of the 1D rotating shallow water system
on one MI355X.

One step = one persistent launch that runs 64 independent parareal solves of
uneven size to completion (the mixed-batch workload, the largest single-GPU
configuration):
    64 problems drawn by default_rng(4): N ~ U{128, 256, 512, 1024},
    eps ~ U{0.1, 0.01, 0.001}, slices ~ U{16..256}; T = 1, K = 8,
    fine ETDRK4 dt = eps/20, M = 32 averaging samples, T0 = dT/eps,
    nu by grid size (3e-5, 1e-5, 1e-6, 1e-7), seeded k^-2 initial spectra up
    to k = N/8 with max|h| = 0.1; FP32 propagators with FP64 correction.
Each solve is the coarse initial sweep plus K iterations of [fine ETDRK4 over
every slice, serial coarse sweep with the FP64 correction, residual]; all of
them run as one dependency graph in one launch.  Inputs are resident on the
device before timing starts.

Metric: fine grid-point-steps per second of whole-step wall time, counting
the fine slices actually computed (K x slices x fine steps x N per solve,
less the K(K-1)/2 slices that earlier iterations made exact and that are
copied instead of recomputed).  The JSON line also carries:
  roofline      the persistent kernel's algorithmic flops per launch over its
                event-timed average duration, against the FP32 vector peak;
  c3            the N = 1024, 256-slice single solve (FP32 propagators with
                FP64 correction), measured the same way;
  fine_batch    the fine propagator alone in its throughput form;
  serving       the request loop (continuous batching) against the plain
                per-request FP64 path, closed and open loop, with sampled
                requests re-run alone and compared with their served results;
  cpu_baseline  the FP64 oracle on the host's cores (a process per problem)
                over a bounded sample of the same workload, timed before the
                GPU is touched.

    python bench.py [--steps K] [--warmup W] [--workload c4|c1|c2|c3]
                    [--no-cpu-baseline] [--no-c3] [--serve-requests R]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MIXED_NAME = "rsw-mixed64-n128-1024-fp32c64"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the C3 measurement beside the headline")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the open-loop serving measurement (0 skips serving)")
    ap.add_argument("--graph", action="store_true",
                    help="replay each step from a captured hipGraph (the pipeline timing then covers the "
                         "whole replay, boundary kernels included)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the schedule autotuner (analytic job durations, default mapping)")
    ap.add_argument("--fine-batch", type=int, default=20480,
                    help="slices of the fine-batch throughput measurement (0 skips it)")
    ap.add_argument("--fine-batch-only", action="store_true",
                    help="only run the fine-batch throughput measurement and print its object")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB three times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def host_workers() -> int:
    """Worker processes for the CPU baseline: the cores this process may run
    on, at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def fine_batch_measure(slices):
    """Throughput form of the fine propagator: aparareal_fine_batch over
    `slices` independent N = 256 FP32 slices of the C2 shape (63 ETDRK4 steps
    each).  The configuration (workgroup shape and FFT plan) is first chosen
    by the fine-batch autotuner on the same states; then three launches are
    timed on the fine kernel alone with HIP events."""
    import numpy as np
    import torch

    from paper_1303_6615_amd import metrics
    from paper_1303_6615_amd.binding import Context, fft_plan
    from paper_1303_6615_amd.inputs import C2, seeded_state

    cfg = C2
    dT = cfg.T / cfg.slices
    u = np.stack([seeded_state(cfg.nx, cfg.k_ic, 1000 + i) for i in range(min(slices, 64))])
    u = torch.tensor(np.resize(u, (slices, 3, cfg.nx)), device="cuda")
    out = torch.empty_like(u)
    with Context(cfg.nx, cfg.eps, cfg.F, cfg.nu) as ctx:
        best, cand_ms = ctx.autotune_fine(u, dT, cfg.fine_steps, precision=0)
        shape, threads, per_wg = ctx.fine_shape(0)
        ctx.fine_batch(u, dT, cfg.fine_steps, precision=0, out=out)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(3):
            ctx.fine_batch(u, dT, cfg.fine_steps, precision=0, out=out)
        torch.cuda.synchronize()
        n, ms = ctx.profile_read()["fine"]
        ctx.profile(False)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite fine batch")
    avg_s = ms / n * 1e-3
    gp = slices * cfg.fine_steps * cfg.nx
    flops = metrics.fine_flops(cfg.nx, slices, cfg.fine_steps)
    return {"workload": f"rsw-n256-eps1e-2 fine batch, {slices} slices x {cfg.fine_steps} ETDRK4 steps, fp32",
            "kernel": f"k_fine<float,256,{threads},{shape // 3}>", "avg_launch_ms": round(avg_s * 1e3, 4),
            "value": round(gp / avg_s, 1), "unit": "fine grid-point-steps/s",
            "tuned_shape": {"config": shape, "shape": shape % 3, "threads": threads, "slices_per_workgroup": per_wg,
                            "fft_plan": fft_plan(cfg.nx, shape // 3),
                            "candidate_ms": [round(x, 4) for x in cand_ms]},
            "roofline": {"bound": "alu", "achieved": round(flops / avg_s / 1e12, 4),
                         "peak": metrics.PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flops / avg_s / 1e12 / metrics.PEAK_FP32_TFLOPS, 4),
                         "frac_of_unpacked_fp32": round(flops / avg_s / 1e12 / metrics.PEAK_FP32_NOPACK_TFLOPS, 4)}}


def _oracle_solve(cfg):
    """One oracle solve in a worker process (BLAS and FFT single-threaded);
    returns its wall time."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        U, _, _ = O.parareal_solve(cfg.initial_state(), cfg.nx, cfg.eps, cfg.F, cfg.nu, cfg.T,
                                   cfg.slices, cfg.K, cfg.fine_steps, cfg.Mbar, cfg.window)
        dt = time.perf_counter() - t0
    assert np.all(np.isfinite(U))
    return dt


def cpu_baseline_mixed(slices=16):
    """The FP64 oracle on every problem of the mixed batch, each cut to its
    first `slices` slices (same dT, fine steps, K and M, so the same per-slice
    work and fine/coarse mix), one process per problem on the host's cores.
    Counted like the GPU: fine grid-point-steps of the slices that are not
    exact copies, over the wall time of the whole pool."""
    import dataclasses
    import multiprocessing as mp

    from paper_1303_6615_amd import metrics
    from paper_1303_6615_amd.inputs import mixed_batch

    probs = []
    for c in mixed_batch(64):
        ns = min(c.slices, slices)
        probs.append(dataclasses.replace(c, slices=ns, T=c.dT * ns))
    workers = host_workers()
    gp = sum(metrics.pipelined_work(c.nx, c.slices, c.K, c.fine_steps, c.Mbar)[0] for c in probs)
    order = sorted(probs, key=lambda c: -c.slices * c.fine_steps * c.nx)     # longest first
    ctx = mp.get_context("fork")           # before any GPU use: plain forks of this process
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_oracle_solve, order, chunksize=1)
    wall = time.perf_counter() - t0
    return {"value": round(gp / wall, 1), "unit": "fine grid-point-steps/s", "cores": workers,
            "kind": "oracle", "seconds": round(wall, 3), "cpu_seconds": round(sum(per), 3),
            "sample": f"all 64 problems of {MIXED_NAME}, each cut to its first {slices} slices "
                      f"(same dT, fine steps, K = 8, M = 32); numpy FP64, one single-threaded "
                      f"process per problem, {workers} at a time"}


def cpu_baseline(cfg):
    """The FP64 oracle on one full solve of the workload, BLAS limited to one thread."""
    dt = _oracle_solve(cfg)
    return {"value": round(cfg.fine_gp_steps() / dt, 1), "unit": "fine grid-point-steps/s", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"one full parareal solve of {cfg.name} (numpy FP64, single thread)"}


def kernel_source_hash():
    """sha256 over the kernel sources and build flags (identifies the kernels that
    a stored counter measurement belongs to)."""
    import hashlib
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_1303_6615_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        h.update(f.encode())
        with open(os.path.join(cs, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_1303_6615_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by a plain copy), or None when there is no
    measurement for this workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic-{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["traffic_bytes"]


def copy_probe(mib):
    """Three plain device-to-device copies of `mib` MiB: each dispatch reads and
    writes exactly mib * 1024 KiB, the yardstick for the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_kib_per_dispatch": mib * 1024, "dispatches": 3}), flush=True)


def measure(W, steps, warmup):
    """Times `steps` steps of workload W after `warmup` untimed ones: wall
    time between two device synchronisations, and the persistent kernel's
    launches from HIP events on the stream it runs on."""
    import torch

    from paper_1303_6615_amd import metrics

    for _ in range(warmup):
        W["step"]()
    torch.cuda.synchronize()
    owner = W["owner"]
    owner.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        W["step"]()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = owner.profile_read()
    owner.profile(False)
    W["check"]()
    kern = {}
    tot_ms = sum(ms for (_, ms) in prof.values())
    for name, (n, ms) in prof.items():
        if n == 0:
            continue
        d = {"launches": n, "avg_ms": round(ms / n, 5), "share": round(ms / tot_ms, 4)}
        if name == "pipeline":
            d["tflops"] = round(W["pipeline_flops"] / (ms / n * 1e-3) / 1e12, 4)
        kern[name] = d
    n_launch, ms_total = prof["pipeline"]
    avg_s = ms_total / n_launch * 1e-3
    achieved = W["pipeline_flops"] / avg_s / 1e12
    fp32 = W["precision"] == 0
    peak = metrics.PEAK_FP32_TFLOPS if fp32 else metrics.PEAK_FP64_TFLOPS
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 6), "traffic": measured_traffic(W["name"]),
                "kernel": W["kernel"], "flops_per_launch": W["pipeline_flops"],
                "avg_launch_ms": round(avg_s * 1e3, 5)}
    return {"value": W["gp_steps"] * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
            "roofline": roofline, "kernels": kern, "dtype": "f32" if fp32 else "f64"}


def _add_measured_frac(roof, peaks):
    """The achieved rate also as a fraction of the vector rate measured on this
    device (FP32 without packed instructions, as the library is built)."""
    key = "fp32_tflops" if roof["peak"] > 100 else "fp64_tflops"
    roof["measured_peak"] = round(peaks[key], 3)
    roof["frac_of_measured_peak"] = round(roof["achieved"] / peaks[key], 4)


def main():
    args = parse()
    if args.copy_mib:
        copy_probe(args.copy_mib)
        return
    if args.fine_batch_only:
        print(json.dumps({"fine_batch": fine_batch_measure(args.fine_batch or 20480)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the parallel-in-time "
              "dimension is the batch dimension of the single-GPU kernels, and this build "
              "uses no second GPU.", file=sys.stderr)
        sys.exit(2)

    # the oracle first: its worker processes are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "c4":
            cpu = cpu_baseline_mixed()
        else:
            from paper_1303_6615_amd.inputs import C1, C2, C3
            cpu = cpu_baseline({"c1": C1, "c2": C2, "c3": C3}[args.workload])
        print(f"# cpu baseline done in {cpu['seconds']} s", file=sys.stderr, flush=True)

    import torch

    from paper_1303_6615_amd.binding import measure_peaks
    torch.cuda.set_device(0)
    peaks = measure_peaks()
    W = single_workload(args, args.workload) if args.workload != "c4" else batch_workload(args)
    m = measure(W, args.steps, args.warmup)
    _add_measured_frac(m["roofline"], peaks)
    line = {
        "metric": "fine grid-point-steps/s at 1 GPU",
        "value": round(m["value"], 1),
        "unit": "fine grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": m["dtype"],
        "data": "synthetic",
        "config": W["config"],
        "roofline": m["roofline"],
        "kernels": m["kernels"],
        "final_residual": W["final_residual"](),
        "autotune": W["autotune"],
        "measured_peaks": {k: round(v, 3) for k, v in peaks.items()},
    }
    W["close"]()
    print("# headline done", file=sys.stderr, flush=True)
    if args.workload == "c4" and not args.no_c3:
        W3 = single_workload(args, "c3")
        m3 = measure(W3, 5, 1)
        _add_measured_frac(m3["roofline"], peaks)
        line["c3"] = {"workload": W3["name"], "value": round(m3["value"], 1), "unit": "fine grid-point-steps/s",
                      "ms_per_solve": round(m3["ms_per_step"], 4), "roofline": m3["roofline"],
                      "final_residual": W3["final_residual"](), "autotune": W3["autotune"]}
        W3["close"]()
        print("# c3 done", file=sys.stderr, flush=True)
    if args.fine_batch > 0:
        line["fine_batch"] = fine_batch_measure(args.fine_batch)
        _add_measured_frac(line["fine_batch"]["roofline"], peaks)
        print("# fine batch done", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        from paper_1303_6615_amd import serving
        line["serving"] = serving.run(n_requests=args.serve_requests, warmup=8)
        print("# serving done", file=sys.stderr, flush=True)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def single_workload(args, which):
    """One parareal solve per step (workloads c1-c3)."""
    import numpy as np
    import torch

    from paper_1303_6615_amd import metrics
    from paper_1303_6615_amd.binding import Context, autotune
    from paper_1303_6615_amd.inputs import C1, C2, C3

    cfg = {"c1": C1, "c2": C2, "c3": C3}[which]
    ctx = Context(cfg.nx, cfg.eps, cfg.F, cfg.nu)
    u0 = torch.tensor(cfg.initial_state(), device="cuda")
    out = torch.empty((cfg.slices + 1, 3, cfg.nx), dtype=torch.float64, device="cuda")
    resid = torch.empty((cfg.K,), dtype=torch.float64, device="cuda")

    def step():
        ctx.solve(u0, cfg.T, cfg.slices, cfg.K, cfg.dt, cfg.Mbar, precision=cfg.precision, out=out, resid=resid)

    ctx.set_option(3, 1 if args.graph else 0)          # AP_OPT_GRAPH

    tuned = None
    if not args.no_autotune:
        # untimed: measures job durations on the device and picks the mapping
        ms = autotune([(ctx, u0, dict(T=cfg.T, slices=cfg.slices, K=cfg.K, dt_fine=cfg.dt, M=cfg.Mbar))],
                      precision=cfg.precision)
        tuned = {"best_ms": round(ms, 4), "split_coarse": ctx.get_option(0), "group_size": ctx.get_option(1),
                 "handoff_us": ctx.get_option(10) / 1000.0}

    def check():
        if not np.all(np.isfinite(resid.cpu().numpy())) or not np.all(np.isfinite(out.cpu().numpy())):
            raise SystemExit("non-finite result")

    gp, work = metrics.pipelined_work(cfg.nx, cfg.slices, cfg.K, cfg.fine_steps, cfg.Mbar)
    typ = "float" if cfg.precision == 0 else "double"
    return {
        "name": cfg.name, "cfg": cfg, "owner": ctx, "step": step, "check": check, "precision": cfg.precision,
        # fine slices and coarse steps actually computed (exact slices are copied)
        "gp_steps": gp,
        "pipeline_flops": work,
        "kernel": f"k_pipeline<{typ},{cfg.nx}>",
        "config": {"workload": cfg.name, "N": cfg.nx, "eps": cfg.eps, "nu": cfg.nu, "F": cfg.F,
                   "T": cfg.T, "slices": cfg.slices, "K": cfg.K, "fine_steps": cfg.fine_steps,
                   "M_avg": cfg.Mbar, "T0": cfg.window,
                   "precision": "fp32 propagators, fp64 correction" if cfg.precision == 0 else "fp64",
                   "parallelism": "time slices as batch, 1 GPU", "graph": bool(args.graph)},
        "final_residual": lambda: float(resid[-1].item()) if cfg.K else None,
        "autotune": tuned,
        "close": ctx.close,
    }


def batch_workload(args):
    """64 uneven problems (N 128-1024, eps 0.1-0.001, 16-256 slices, K = 8) in
    one persistent launch per step."""
    import numpy as np
    import torch

    from paper_1303_6615_amd import metrics
    from paper_1303_6615_amd.binding import Context, _batch_items, _check, _stream, autotune, lib
    from paper_1303_6615_amd.inputs import mixed_batch

    probs = mixed_batch(64)
    ctxs = [Context(c.nx, c.eps, c.F, c.nu) for c in probs]
    items = [(x, torch.tensor(c.initial_state(), device="cuda"),
              dict(T=c.T, slices=c.slices, K=c.K, dt_fine=c.dt, M=c.Mbar)) for x, c in zip(ctxs, probs)]
    arr, outs = _batch_items(items, 0)
    ctxs[0].set_option(3, 1 if args.graph else 0)      # AP_OPT_GRAPH (the first item owns the launch)

    def step():
        _check(lib().aparareal_solve_batch(arr, len(items), _stream(torch)))

    tuned = None
    if not args.no_autotune:
        ms = autotune(items, precision=0)
        tuned = {"best_ms": round(ms, 4), "split_coarse": ctxs[0].get_option(0),
                 "group_sizes": sorted({c.get_option(1) for c in ctxs}), "handoff_us": ctxs[0].get_option(10) / 1000.0}

    def check():
        for U, r, _ in outs:
            if not np.all(np.isfinite(r.cpu().numpy())) or not np.all(np.isfinite(U.cpu().numpy())):
                raise SystemExit("non-finite result")

    work = [metrics.pipelined_work(c.nx, c.slices, c.K, c.fine_steps, c.Mbar) for c in probs]
    flops = sum(w[1] for w in work)

    def close():
        for x in ctxs:
            x.close()

    return {
        "name": MIXED_NAME, "cfg": None, "owner": ctxs[0], "step": step, "check": check,
        "precision": 0, "gp_steps": sum(w[0] for w in work), "pipeline_flops": flops,
        "kernel": "k_pipeline<float,64,128,256,512,1024>",
        "config": {"workload": MIXED_NAME, "problems": len(probs),
                   "N": sorted({c.nx for c in probs}), "eps": sorted({c.eps for c in probs}),
                   "slices": [min(c.slices for c in probs), max(c.slices for c in probs)], "K": 8, "T": 1.0,
                   "M_avg": 32, "precision": "fp32 propagators, fp64 correction",
                   "parallelism": "problems x time slices as batch, 1 GPU", "graph": bool(args.graph)},
        "final_residual": lambda: max(float(r[-1].item()) for _, r, _ in outs),
        "autotune": tuned,
        "close": close,
    }


if __name__ == "__main__":
    main()
