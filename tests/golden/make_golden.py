"""Writes the stored oracle results used by the full-size GPU parity tests.

    python tests/golden/make_golden.py [--jobs J] [--only c1,c2,c3,c4]

Every value written here comes from the FP64 oracle (`oracle.parareal_solve`,
the parareal iteration of eq. HMM parareal iteration / Alg. 4 with the ETDRK4
fine solver of Sec. 6.2 and the asymptotic coarse step of Alg. 2) on the seeded
initial states of `paper_1303_6615_amd.inputs`; nothing comes from the HIP
path.  The solves are independent, so they run in a process pool, each
single-threaded.

Files (numpy .npz, no pickles):
  solve_<workload>.npz   the single-solve workloads:
      U      complex128 [Ns+1, 3, Kd+1]  the final iterate U^K, retained modes
             (the oracle's spectral convention; modes above Kd are exactly 0)
      r      float64 [K]                 the residuals r^1..r^K
  mixed64.npz            the 64-problem mixed batch:
      p<i>_slices  int32 [m]      sampled slice indices of problem i
      p<i>_U       complex64 [m, 3, Kd+1]  U^K at those slices (rounded to
                                  complex64 for size: 6e-8 relative, far
                                  below the 2e-5 tolerance it is checked at)
      p<i>_r       float64 [K]    the residuals of problem i
The sampled slices of problem i are 1, Ns/3, 2Ns/3, Ns and four more drawn by
numpy.random.default_rng(7000 + i); all 64 problems are covered.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def mixed_slices(ns: int, i: int) -> np.ndarray:
    """Sampled slice indices of problem i of the mixed batch (Ns slices)."""
    rng = np.random.default_rng(7000 + i)
    fixed = {1, max(1, ns // 3), max(1, 2 * ns // 3), ns}
    extra = set(int(v) for v in rng.choice(np.arange(1, ns + 1), size=min(4, ns), replace=False))
    return np.array(sorted(fixed | extra), dtype=np.int32)


def _solve(cfg):
    from threadpoolctl import threadpool_limits

    import oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, resid, hist = O.parareal_solve(cfg.initial_state(), cfg.nx, cfg.eps, cfg.F, cfg.nu, cfg.T, cfg.slices,
                                          cfg.K, cfg.fine_steps, cfg.Mbar, cfg.window)
        dt = time.perf_counter() - t0
    kp = cfg.nx // 3 + 1
    return cfg.name, hist[-1][:, :, :kp], np.asarray(resid, dtype=np.float64), dt


def main() -> None:
    from paper_1303_6615_amd.inputs import C1, C2, C3, mixed_batch

    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="c1,c2,c3,c4")
    args = ap.parse_args()
    which = set(args.only.split(","))
    single = {"c1": C1, "c2": C2, "c3": C3}
    mixed = mixed_batch() if "c4" in which else []
    work = [single[w] for w in ("c3", "c2", "c1") if w in which] + mixed
    cost = {id(c): c.K * c.slices * c.fine_steps * c.nx + 4 * (c.K + 1) * c.slices * c.Mbar * c.nx for c in work}
    work.sort(key=lambda c: -cost[id(c)])          # longest first
    results = {}
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for name, U, r, dt in ex.map(_solve, work):
            results[name] = (U, r)
            print(f"{name}: {dt:.1f} s", flush=True)
    for w, cfg in single.items():
        if w in which:
            U, r = results[cfg.name]
            np.savez(os.path.join(HERE, f"solve_{cfg.name}.npz"), U=U, r=r)
    if mixed:
        arrs = {}
        for i, cfg in enumerate(mixed):
            U, r = results[cfg.name]
            sl = mixed_slices(cfg.slices, i)
            arrs[f"p{i}_slices"] = sl
            arrs[f"p{i}_U"] = U[sl].astype(np.complex64)
            arrs[f"p{i}_r"] = r
        np.savez(os.path.join(HERE, "mixed64.npz"), **arrs)


if __name__ == "__main__":
    main()
