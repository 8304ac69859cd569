"""Algorithmic work counts and MI355X peaks used for roofline reporting.

Counts are what the method must compute, independent of how a kernel does it:
full-length FFTs (the products need every grid value) at the conventional
2.5 n log2 n flops per real transform, ~7 pointwise flops per grid value per
nonlinear evaluation, and the per-wavenumber 3x3 complex linear algebra on
the retained modes only.

  fine grid-point-step (one ETDRK4 step, one grid value):
      Phi(N) = 4 [6 * 2.5 log2 N + 7] + 696 (Kd + 1) / N
      (4 nonlinear evaluations of 6 real FFTs; 9 complex 3x3 mat-vecs = 648 and
       ~48 vector flops per retained mode per step)
  coarse step (Alg. 2, M averaging samples, M-1 with nonzero weight):
      2 (M - 1) [6 * 2.5 N log2 N + 7 N + 144 (Kd + 1)]
      (two averaged evaluations; each sample rotates in and out with a 3x3
       complex mat-vec per retained mode, 2 * 72 flops)
"""
from __future__ import annotations

import math

# MI355X published peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
# = 78.6 TFLOP/s for FP64 and for non-packed FP32; packed FP32 doubles the FP32
# rate to 157.3 TFLOP/s.  HBM3E 8 TB/s.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NOPACK_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
CUS = 256
CLOCK_GHZ = 2.4


def kd(nx: int) -> int:
    return nx // 3


def fine_flops_per_gp_step(nx: int) -> float:
    """Phi(N): algorithmic flops per fine grid-point-step."""
    return 4.0 * (6 * 2.5 * math.log2(nx) + 7) + 696.0 * (kd(nx) + 1) / nx


def fine_flops(nx: int, slices: int, steps: int) -> float:
    """Flops of one fine-batch launch over `slices` states x `steps` steps."""
    return fine_flops_per_gp_step(nx) * nx * slices * steps


def coarse_step_flops(nx: int, M: int) -> float:
    """Algorithmic flops of one asymptotic coarse step with M samples."""
    per_eval = 6 * 2.5 * nx * math.log2(nx) + 7 * nx + 144.0 * (kd(nx) + 1)
    return 2.0 * (M - 1) * per_eval


def sweep_flops(nx: int, M: int, slices: int) -> float:
    """Flops of one serial sweep (one coarse step per slice)."""
    return coarse_step_flops(nx, M) * slices


def state_bytes_modal(nx: int) -> int:
    """FP64 modal state: 3 fields x (Kd+1) complex doubles."""
    return 3 * (kd(nx) + 1) * 16


def pipelined_work(nx: int, slices: int, K: int, steps: int, M: int, skip: bool = True):
    """(fine grid-point-steps, algorithmic flops) of one pipelined solve.

    With slice skipping, iteration k+1 does not re-run the fine slices n <= k
    (exact after k iterations) and copies their coarse steps: K(K-1)/2 fine
    slices and K(K+1)/2 coarse steps fewer when slices >= K.  Only the work
    actually done is counted."""
    fine_slices = sum(max(0, slices - (k if skip else 0)) for k in range(K))
    coarse_steps = slices + sum(max(0, slices - (k if skip else 0)) for k in range(1, K + 1))
    gp = fine_slices * steps * nx
    flops = fine_flops(nx, fine_slices, steps) + coarse_step_flops(nx, M) * coarse_steps
    return gp, flops
