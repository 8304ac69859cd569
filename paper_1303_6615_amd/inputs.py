"""Seeded synthetic initial states and the workload parameter sets.

This module holds no arithmetic of the method: it only draws random Fourier
series and lists parameters.  Both the oracle and the GPU path receive the
arrays it returns.

Initial state recipe (the paper's own initial condition, eq. initial condition
in Sec. 6.2, is a fixed analytic height bump; the workloads here use seeded
random spectra of the same smoothness class instead):

    rng = numpy.random.default_rng(seed)
    z = rng.standard_normal((3, K_ic, 2))
    fhat_k = k^-2 (z[f, k-1, 0] + i z[f, k-1, 1]),  1 <= k <= K_ic,  fhat_0 = 0
    f(x_j) = sum_k 2 Re(fhat_k exp(i k x_j)),  x_j = 2 pi j / Nx
    all three fields scaled by one factor so that max_j |h(x_j)| = 0.1
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def seeded_state(nx: int, k_ic: int, seed: int, amplitude: float = 0.1) -> np.ndarray:
    """Random k^-2 Fourier series for (v1, v2, h) on the grid, float64 [3, Nx]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((3, k_ic, 2))
    k = np.arange(1, k_ic + 1, dtype=np.float64)
    x = 2.0 * np.pi * np.arange(nx, dtype=np.float64) / nx
    phase = np.outer(k, x)                                  # [K_ic, Nx]
    cos, sin = np.cos(phase), np.sin(phase)
    out = np.empty((3, nx), dtype=np.float64)
    for f in range(3):
        re = z[f, :, 0] / k ** 2
        im = z[f, :, 1] / k ** 2
        # 2 Re((re + i im)(cos + i sin)) = 2 (re cos - im sin)
        out[f] = 2.0 * (re @ cos - im @ sin)
    scale = amplitude / np.max(np.abs(out[2]))
    return out * scale


def paper_height_state(nx: int) -> np.ndarray:
    """The paper's analytic initial condition (eq. initial condition, Sec. 6.2):
    v1 = v2 = 0, h = c1 (exp(-4(x-pi/2)^2) sin(3(x-pi/2)) + exp(-2(x-pi)^2) sin(8(x-pi))) + c0
    with c0 removing the mean and c1 setting max|h| = 1 (the text's "c1 and c2"
    is read as c1 and c0)."""
    x = 2.0 * np.pi * np.arange(nx, dtype=np.float64) / nx
    g = (np.exp(-4.0 * (x - np.pi / 2) ** 2) * np.sin(3.0 * (x - np.pi / 2))
         + np.exp(-2.0 * (x - np.pi) ** 2) * np.sin(8.0 * (x - np.pi)))
    g = g - g.mean()
    h = g / np.max(np.abs(g))
    out = np.zeros((3, nx), dtype=np.float64)
    out[2] = h
    return out


PREC_FP32 = 0   # FP32 propagators, FP64 parareal correction
PREC_FP64 = 1   # everything FP64


@dataclass
class SolveConfig:
    """One parareal solve of the RSW system on the periodic grid."""
    name: str
    nx: int
    eps: float
    nu: float
    T: float
    slices: int
    K: int
    dt: float
    Mbar: int
    k_ic: int
    seed: int
    F: float = 1.0
    T0: float | None = None            # fast-time window; None -> dT/eps
    precision: int = PREC_FP32

    @property
    def dT(self) -> float:
        return self.T / self.slices

    @property
    def fine_steps(self) -> int:
        return max(1, int(math.ceil(self.dT / self.dt - 1e-9)))

    @property
    def window(self) -> float:
        return self.dT / self.eps if self.T0 is None else self.T0

    def initial_state(self) -> np.ndarray:
        return seeded_state(self.nx, self.k_ic, self.seed)

    def fine_gp_steps(self) -> int:
        """Fine grid-point-steps of one solve: K * slices * fine_steps * Nx."""
        return self.K * self.slices * self.fine_steps * self.nx


# Single-solve workloads: N = 64 FP64 (small), N = 256 and N = 1024 (FP32 propagators).
C1 = SolveConfig("rsw-n64-eps1e-2-s16-k5-fp64", nx=64, eps=0.01, nu=1e-4, T=1.0,
                 slices=16, K=5, dt=0.01 / 20, Mbar=16, k_ic=8, seed=1,
                 precision=PREC_FP64)
C2 = SolveConfig("rsw-n256-eps1e-2-s64-k8-fp32c64", nx=256, eps=0.01, nu=1e-5, T=2.0,
                 slices=64, K=8, dt=0.01 / 20, Mbar=32, k_ic=32, seed=2,
                 precision=PREC_FP32)
C3 = SolveConfig("rsw-n1024-eps1e-3-s256-k10-fp32c64", nx=1024, eps=0.001, nu=1e-7,
                 T=1.0, slices=256, K=10, dt=0.001 / 10, Mbar=64, k_ic=128, seed=3,
                 precision=PREC_FP32)

# Hyperviscosity per grid size for the mixed workloads: interpolates the three
# single-solve workloads up to N = 1024.  At N = 2048 a smaller value than
# 1e-6 lets the explicit midpoint coarse step (Alg. 2) diverge on some
# requests of the serving stream (velocities up to ~0.6 with slices of
# ~T/32): with 1e-8 four of 184 drawn requests diverge in the FP64 oracle
# and on the GPU alike, with 1e-7 one, with 1e-6 none.
NU_BY_NX = {64: 1e-4, 128: 3e-5, 256: 1e-5, 512: 1e-6, 1024: 1e-7, 2048: 1e-6}


def mixed_batch(count: int = 64, seed: int = 4, nxs=(128, 256, 512, 1024),
                epss=(0.1, 0.01, 0.001), slice_range=(16, 256), K: int = 8,
                T: float = 1.0, Mbar: int = 32) -> list[SolveConfig]:
    """Uneven independent problems for one batched launch (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.choice(nxs))
        eps = float(rng.choice(epss))
        ns = int(rng.integers(slice_range[0], slice_range[1] + 1))
        out.append(SolveConfig(f"mix{i}", nx=nx, eps=eps, nu=NU_BY_NX[nx], T=T,
                               slices=ns, K=K, dt=eps / 20, Mbar=Mbar, k_ic=nx // 8,
                               seed=4000 + i, precision=PREC_FP32))
    return out


def serving_requests(count: int, seed: int = 5, nxs=(128, 256, 512, 1024, 2048),
                     epss=(0.1, 0.01, 0.001), T_range=(0.5, 4.0), K: int = 8,
                     Mbar: int = 32) -> list[SolveConfig]:
    """Request stream for the serving loop: sizes drawn like the mixed batch,
    T ~ U[0.5, 4], slices = clamp(2^round(log2(32 T)), 16, 256)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.choice(nxs))
        eps = float(rng.choice(epss))
        T = float(rng.uniform(*T_range))
        ns = int(min(256, max(16, 2 ** int(round(math.log2(32.0 * T))))))
        out.append(SolveConfig(f"req{i}", nx=nx, eps=eps, nu=NU_BY_NX[nx], T=T,
                               slices=ns, K=K, dt=eps / 20, Mbar=Mbar, k_ic=nx // 8,
                               seed=5000 + i, precision=PREC_FP32))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 55) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
