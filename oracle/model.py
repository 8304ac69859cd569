"""The paper's parallel-speedup estimate (Sec. 5, eq. speedup upper bound).

With N slices, M fine steps per slice, nu iterations, tau_f the wall time of
one fine step and tau_c that of one coarse step, the estimated speedup of the
parareal solve over the serial fine integration is

    tau_f N M / (nu (tau_f M + tau_c N + tau_c) + tau_c N).

Sec. 6.2 evaluates it with tau_c = tau_f and drops the lone tau_c term
(its printed expression N (dT/dt) / (5 ((dT/dt) + N) + N)).
"""


def estimated_speedup(N: float, M: float, iterations: float,
                      tau_f: float = 1.0, tau_c: float = 1.0,
                      include_lone_coarse: bool = True) -> float:
    """Speedup of Sec. 5; `include_lone_coarse=False` gives the Sec. 6.2 form."""
    lone = tau_c if include_lone_coarse else 0.0
    return tau_f * N * M / (iterations * (tau_f * M + tau_c * N + lone) + tau_c * N)


def speedup_upper_bound(N: float, M: float, iterations: float,
                        tau_f: float = 1.0, tau_c: float = 1.0) -> float:
    """Right-hand side of eq. speedup upper bound: min(tau_f/tau_c * M/(nu+1), N/nu)."""
    return min(tau_f / tau_c * M / (iterations + 1), N / iterations)
