"""ctypes binding of libaparareal.so (argument marshalling only).

Every array is a torch CUDA tensor (float64, contiguous) whose device pointer is
handed to the library together with torch's current stream; all computation
happens in the library's HIP kernels.  The library must be built
(``python -m paper_1303_6615_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

from .build import LIB_PATH, ROOT

HEADER = os.path.join(ROOT, "include", "aparareal.h")

AP_OK, AP_PENDING = 0, 1
AP_PREC_FP32, AP_PREC_FP64 = 0, 1
ERRORS = {-1: "AP_EINVAL", -2: "AP_ENOMEM", -3: "AP_EDEVICE", -4: "AP_ENOTFOUND",
          -5: "AP_ENUMERIC", -6: "AP_EBUSY"}


class APError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("slices", ctypes.c_int), ("K", ctypes.c_int),
                ("dt_fine", ctypes.c_double), ("M_avg", ctypes.c_int), ("T0", ctypes.c_double),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int)]


class BatchItem(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("u0", ctypes.c_void_p), ("params", SolveParams),
                ("U_out", ctypes.c_void_p), ("resid", ctypes.c_void_p)]


AP_OPT_SPLIT, AP_OPT_GROUP, AP_OPT_GRID, AP_OPT_GRAPH, AP_OPT_SKIP, AP_OPT_SWEEPS = 0, 1, 2, 3, 4, 5
AP_OPT_FINE, AP_OPT_COARSE, AP_OPT_FINE_GROUP, AP_OPT_FINE_SHAPE, AP_OPT_HANDOFF_NS = 6, 7, 8, 9, 10
AP_FINE_CONFIGS = 6
JOB_COARSE, JOB_FINE, JOB_STAGE1, JOB_STAGE2, JOB_COPY = 0, 1, 2, 3, 4


_lib = None
_vp, _dp, _i, _d = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double

_SIGNATURES = {
    "aparareal_last_error": (ctypes.c_char_p, []),
    "aparareal_create": (_vp, [_i, _d, _d, _d]),
    "aparareal_destroy": (_i, [_vp]),
    "aparareal_nonlinear": (_i, [_vp, _dp, _dp, _i, _i, _vp]),
    "aparareal_fine_batch": (_i, [_vp, _dp, _dp, _i, _d, _i, _i, _vp]),
    "aparareal_fine_batch_noalloc": (_i, [_vp, _dp, _dp, _i, _d, _i, _i, _vp]),
    "aparareal_strang_batch": (_i, [_vp, _dp, _dp, _i, _d, _i, _i, _vp]),
    "aparareal_average": (_i, [_vp, _dp, _dp, _i, _d, _i, _i, _vp]),
    "aparareal_coarse": (_i, [_vp, _dp, _dp, _i, _d, _i, _d, _i, _vp]),
    "aparareal_solve": (_i, [_vp, _dp, ctypes.POINTER(SolveParams), _dp, _dp, _vp]),
    "aparareal_profile": (_i, [_vp, _i]),
    "aparareal_solve_batch": (_i, [ctypes.POINTER(BatchItem), _i, _vp]),
    "aparareal_set_option": (_i, [_vp, _i, _i]),
    "aparareal_autotune": (_i, [ctypes.POINTER(BatchItem), _i, _vp, ctypes.POINTER(_d)]),
    "aparareal_autotune_fine": (_i, [_vp, _dp, _i, _d, _i, _i, _vp, ctypes.POINTER(_d), ctypes.POINTER(_i)]),
    "aparareal_fine_shape": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "aparareal_fft_plan": (_i, [_i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "aparareal_measure_peaks": (_i, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "aparareal_get_option": (_i, [_vp, _i, ctypes.POINTER(_i)]),
    "aparareal_pipeline_schedule": (_i, [_i, ctypes.POINTER(SolveParams), _i, _i, _i, ctypes.POINTER(_i), _i]),
    "aparareal_pipeline_schedule_batch": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(SolveParams), _i, _i, _i,
                                               ctypes.POINTER(_d), ctypes.POINTER(_i), _i]),
    "aparareal_pipeline_status": (_i, [_vp, ctypes.POINTER(_i)]),
    "aparareal_pipeline_trace": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_longlong), _i]),
    "aparareal_profile_read": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "aparareal_serve_create": (_vp, [ctypes.c_size_t, _i]),
    "aparareal_serve_submit": (_i, [_vp, _i, _d, _d, _d, _dp, ctypes.POINTER(SolveParams),
                                    ctypes.POINTER(ctypes.c_ulonglong)]),
    "aparareal_serve_poll": (_i, [_vp, ctypes.c_ulonglong, _dp, _dp, ctypes.POINTER(_d)]),
    "aparareal_serve_stats": (_i, [_vp, ctypes.POINTER(ctypes.c_ulonglong)]),
    "aparareal_serve_destroy": (_i, [_vp]),
}

KERNEL_CLASSES = {0: "fine", 1: "sweep", 2: "to_modal", 3: "to_physical", 4: "resid",
                  5: "nonlinear", 6: "average", 7: "coarse", 8: "pipeline"}


def header_symbols() -> list[str]:
    """Function names declared in include/aparareal.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(aparareal_\w+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; loading it first lets this library's
        # runtime bind to the same HSA runtime (loading this library first
        # leaves torch without a device)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1303_6615_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def pipeline_schedule(N: int, T: float, slices: int, K: int, dt_fine: float, M: int, split: int = -1,
                      group: int = 0, precision: int = AP_PREC_FP32,
                      fine_group: int = 1, tol: float = 0.0) -> list[tuple[int, int, int, int]]:
    """Job order of the pipelined solve as (type, k, n, g) quadruples (host only);
    a fine job (type 1) covers slices n .. n + g - 1."""
    p = SolveParams(float(T), int(slices), int(K), float(dt_fine), int(M), 0.0, float(tol), int(precision))
    cnt = _check(lib().aparareal_pipeline_schedule(N, ctypes.byref(p), split, group, fine_group, None, 0))
    buf = (ctypes.c_int * (4 * max(cnt, 1)))()
    cnt = _check(lib().aparareal_pipeline_schedule(N, ctypes.byref(p), split, group, fine_group, buf, cnt))
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(cnt)]


def pipeline_schedule_batch(problems, split: int = -1, group: int = 0, fine_group: int = 1,
                            precision: int = AP_PREC_FP32, cost=None) -> list[tuple[int, int, int, int, int]]:
    """Job order of a batched pipelined launch (host only) as (prob, type, k, n, g)
    quintuples; problems: (N, T, slices, K, dt_fine, M[, tol]) tuples; cost: optional
    per-problem (fine step, stage 1, stage 2, whole) durations in us."""
    cnt_p = len(problems)
    Ns = (ctypes.c_int * cnt_p)(*[int(q[0]) for q in problems])
    ps = (SolveParams * cnt_p)(*[SolveParams(float(q[1]), int(q[2]), int(q[3]), float(q[4]), int(q[5]), 0.0,
                                             float(q[6]) if len(q) > 6 else 0.0, int(precision))
                                 for q in problems])
    cs = None
    if cost is not None:
        cs = (ctypes.c_double * (4 * cnt_p))(*[float(v) for row in cost for v in row])
    cnt = _check(lib().aparareal_pipeline_schedule_batch(cnt_p, Ns, ps, split, group, fine_group, cs, None, 0))
    buf = (ctypes.c_int * (5 * max(cnt, 1)))()
    cnt = _check(lib().aparareal_pipeline_schedule_batch(cnt_p, Ns, ps, split, group, fine_group, cs, buf, cnt))
    return [tuple(buf[5 * i:5 * i + 5]) for i in range(cnt)]


def _batch_items(problems, precision):
    import torch
    items = (BatchItem * len(problems))()
    outs = []
    for i, (ctx, u0, prm) in enumerate(problems):
        u0 = _states(u0, ctx.N, "u0")
        S, K = int(prm["slices"]), int(prm["K"])
        U = torch.empty((S + 1, 3, ctx.N), dtype=torch.float64, device=u0.device)
        r = torch.empty((max(K, 1),), dtype=torch.float64, device=u0.device)
        items[i].ctx = ctx._h
        items[i].u0 = u0.data_ptr()
        items[i].params = SolveParams(float(prm["T"]), S, K, float(prm["dt_fine"]), int(prm["M"]),
                                      float(prm.get("T0", 0.0)), 0.0, int(precision))
        items[i].U_out = U.data_ptr()
        items[i].resid = r.data_ptr()
        outs.append((U, r[:K], u0))
    return items, outs


def solve_batch(problems, precision: int = AP_PREC_FP32):
    """Many problems in one persistent launch.  `problems` is a list of
    (Context, u0, dict(T, slices, K, dt_fine, M[, T0])); returns a list of
    (U [slices+1, 3, N], resid [K]) CUDA tensors."""
    import torch
    items, outs = _batch_items(problems, precision)
    _check(lib().aparareal_solve_batch(items, len(problems), _stream(torch)))
    return [(U, r) for (U, r, _) in outs]


def autotune(problems, precision: int = AP_PREC_FP32) -> float:
    """Tune the pipelined schedule of these problems (as for solve_batch; one
    problem tunes a single solve).  Returns the best solve time in ms."""
    import torch
    items, outs = _batch_items(problems, precision)
    ms = ctypes.c_double(0.0)
    _check(lib().aparareal_autotune(items, len(problems), _stream(torch), ctypes.byref(ms)))
    torch.cuda.synchronize()
    return ms.value


def fft_plan(N: int, plan: int = 0) -> dict:
    """Radices of FFT plan `plan` for grid size N, and how many exchanges
    between its passes are register row swaps."""
    r = (ctypes.c_int * 4)()
    n, x = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().aparareal_fft_plan(int(N), int(plan), r, ctypes.byref(n), ctypes.byref(x)))
    return {"plan": int(plan), "radices": list(r)[:n.value], "register_exchanges": x.value}


def measure_peaks() -> dict:
    """Measured FP32 / FP64 vector FMA rates (TFLOP/s) and LDS read bandwidth
    (TB/s) of the current device (microbenchmark kernels in the library)."""
    import torch
    a, b, c = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().aparareal_measure_peaks(_stream(torch), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"fp32_tflops": a.value, "fp64_tflops": b.value, "lds_tbps": c.value}


def _check(rc: int) -> int:
    if rc < 0:
        raise APError(rc, lib().aparareal_last_error().decode())
    return rc


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _states(x, n: int, name: str):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.dim() < 2 or x.shape[-2:] != (3, n):
        raise ValueError(f"{name} must have shape [..., 3, {n}], got {tuple(x.shape)}")
    return x


class Context:
    """One library context: grid size N, eps, F, nu on the current device."""

    def __init__(self, N: int, eps: float, F: float = 1.0, nu: float = 0.0):
        self.N, self.eps, self.F, self.nu = int(N), float(eps), float(F), float(nu)
        h = lib().aparareal_create(self.N, self.eps, self.F, self.nu)
        if not h:
            raise APError(-1, lib().aparareal_last_error().decode())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().aparareal_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- batched propagators -------------------------------------------------
    def _batched(self, fn, U, *args, out=None):
        import torch
        U = _states(U, self.N, "U")
        out = torch.empty_like(U) if out is None else _states(out, self.N, "out")
        batch = U.numel() // (3 * self.N)
        _check(fn(self._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  batch, *args, _stream(torch)))
        return out

    def nonlinear(self, U, precision: int = AP_PREC_FP64, out=None):
        return self._batched(lib().aparareal_nonlinear, U, precision, out=out)

    def fine_batch(self, U, dT: float, steps: int, precision: int = AP_PREC_FP32, out=None):
        return self._batched(lib().aparareal_fine_batch, U, float(dT), int(steps), precision, out=out)

    def fine_batch_noalloc(self, U, dT: float, steps: int, precision: int = AP_PREC_FP32, out=None):
        """fine_batch through the entry point that allocates nothing (its
        scratch is the library's per-device array); `out` may be passed in."""
        return self._batched(lib().aparareal_fine_batch_noalloc, U, float(dT), int(steps), precision, out=out)

    def autotune_fine(self, U, dT: float, steps: int, precision: int = AP_PREC_FP32):
        """Time the fine batch's configurations (workgroup shape c % 3, FFT
        plan c // 3) on U, keep and cache the fastest; returns (best
        configuration, [mean ms per configuration, -1 where not compiled])."""
        import torch
        U = _states(U, self.N, "U")
        ms = (ctypes.c_double * AP_FINE_CONFIGS)()
        best = ctypes.c_int(0)
        _check(lib().aparareal_autotune_fine(self._h, ctypes.c_void_p(U.data_ptr()), U.numel() // (3 * self.N),
                                             float(dT), int(steps), int(precision), _stream(torch), ms,
                                             ctypes.byref(best)))
        return best.value, list(ms)

    def fine_shape(self, precision: int = AP_PREC_FP32) -> tuple[int, int, int]:
        """(configuration, threads per workgroup, slices per workgroup) of fine
        batches; configuration c is workgroup shape c % 3 with FFT plan c // 3."""
        sh, nt, j = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().aparareal_fine_shape(self._h, int(precision), ctypes.byref(sh), ctypes.byref(nt),
                                          ctypes.byref(j)))
        return sh.value, nt.value, j.value

    def strang_batch(self, U, dT: float, steps: int, precision: int = AP_PREC_FP32, out=None):
        return self._batched(lib().aparareal_strang_batch, U, float(dT), int(steps), precision, out=out)

    def average(self, U, T0: float, M: int, precision: int = AP_PREC_FP32, out=None):
        return self._batched(lib().aparareal_average, U, float(T0), int(M), precision, out=out)

    def coarse(self, U, dT: float, M: int, T0: float = 0.0, precision: int = AP_PREC_FP32, out=None):
        return self._batched(lib().aparareal_coarse, U, float(dT), int(M), float(T0), precision, out=out)

    # -- kernel timing ----------------------------------------------------------
    def profile(self, enable: bool = True):
        _check(lib().aparareal_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{class name: (launches, total ms)} for every kernel class (syncs)."""
        out = {}
        for cls, name in KERNEL_CLASSES.items():
            n, ms = ctypes.c_int(0), ctypes.c_double(0.0)
            _check(lib().aparareal_profile_read(self._h, cls, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (n.value, ms.value)
        return out

    def pipeline_status(self) -> tuple[int, int, int]:
        """(stalled, job, flag) of the last pipelined solve (synchronises)."""
        buf = (ctypes.c_int * 3)()
        _check(lib().aparareal_pipeline_status(self._h, buf))
        return buf[0], buf[1], buf[2]

    def trace(self, enable: bool):
        """Record per-job device-clock intervals of the following pipelined solves."""
        _check(lib().aparareal_pipeline_trace(self._h, 1 if enable else 0, None, 0))

    def trace_read(self, max_jobs: int = 1 << 20):
        """Last launch's jobs: list of (problem, type, k, n, g, start_tick, end_tick, workgroup)."""
        buf = (ctypes.c_longlong * (8 * max_jobs))()
        n = _check(lib().aparareal_pipeline_trace(self._h, -1, buf, max_jobs))
        return [tuple(buf[8 * i:8 * i + 8]) for i in range(n)]

    def set_option(self, option: int, value: int):
        _check(lib().aparareal_set_option(self._h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int(0)
        _check(lib().aparareal_get_option(self._h, int(option), ctypes.byref(v)))
        return v.value

    # -- the parareal solve ----------------------------------------------------
    def solve(self, u0, T: float, slices: int, K: int, dt_fine: float, M: int, T0: float = 0.0,
              tol: float = 0.0, precision: int = AP_PREC_FP32, out=None, resid=None):
        """Returns (U [slices+1, 3, N], resid [K]) as CUDA float64 tensors."""
        import torch
        u0 = _states(u0, self.N, "u0")
        if u0.numel() != 3 * self.N:
            raise ValueError("u0 must hold one state [3, N]")
        p = SolveParams(float(T), int(slices), int(K), float(dt_fine), int(M), float(T0),
                        float(tol), int(precision))
        if out is None:
            out = torch.empty((slices + 1, 3, self.N), dtype=torch.float64, device=u0.device)
        if resid is None:
            resid = torch.empty((max(K, 1),), dtype=torch.float64, device=u0.device)
        _check(lib().aparareal_solve(self._h, ctypes.c_void_p(u0.data_ptr()), ctypes.byref(p),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(resid.data_ptr()), _stream(torch)))
        return out, resid[:K]


class Server:
    """The library's serving loop (host arrays in and out)."""

    STATS = ("completed", "failed", "queued", "running", "launches", "bytes_held", "peak_bytes")

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        h = lib().aparareal_serve_create(int(hbm_budget_bytes), int(max_slots))
        if not h:
            raise APError(-1, lib().aparareal_last_error().decode())
        self._h = ctypes.c_void_p(h)
        self._shape = {}

    def submit(self, N: int, eps: float, F: float, nu: float, u0, T: float, slices: int, K: int,
               dt_fine: float, M: int, T0: float = 0.0, precision: int = AP_PREC_FP32) -> int:
        import numpy as np
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        if u0.shape != (3, N):
            raise ValueError(f"u0 must have shape (3, {N})")
        p = SolveParams(float(T), int(slices), int(K), float(dt_fine), int(M), float(T0), 0.0, int(precision))
        t = ctypes.c_ulonglong(0)
        _check(lib().aparareal_serve_submit(self._h, int(N), float(eps), float(F), float(nu),
                                            ctypes.c_void_p(u0.ctypes.data), ctypes.byref(p), ctypes.byref(t)))
        self._shape[t.value] = (int(N), int(slices), int(K))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (U [slices+1, 3, N], resid [K], latency_s) as numpy arrays."""
        import numpy as np
        N, S, K = self._shape[ticket]
        U = np.empty((S + 1, 3, N), dtype=np.float64)
        r = np.empty((max(K, 1),), dtype=np.float64)
        lat = ctypes.c_double(0.0)
        rc = lib().aparareal_serve_poll(self._h, ctypes.c_ulonglong(ticket), ctypes.c_void_p(U.ctypes.data),
                                        ctypes.c_void_p(r.ctypes.data), ctypes.byref(lat))
        if rc == AP_PENDING:
            return None
        del self._shape[ticket]
        _check(rc)
        return U, r[:K], lat.value

    def stats(self) -> dict:
        buf = (ctypes.c_ulonglong * 7)()
        _check(lib().aparareal_serve_stats(self._h, buf))
        return dict(zip(self.STATS, list(buf)))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().aparareal_serve_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
