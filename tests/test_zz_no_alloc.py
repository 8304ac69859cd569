"""The fine batch through the entry point that allocates nothing
(aparareal_fine_batch_noalloc, scratch in the library's per-device array)
against the ordinary entry point (aparareal_fine_batch), through the C ABI:
identical bits on two calls in a row, the second with a smaller batch and a
different step size, and within the precision's tolerance of the FP64 oracle
(Cox-Matthews ETDRK4, the fine solver of Sec. 6.2)."""
import numpy as np
import pytest

import oracle as O
from paper_1303_6615_amd.inputs import NU_BY_NX, seeded_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("n,eps,prec,tol", [(256, 0.01, 0, 2e-5), (1024, 0.001, 1, 1e-11), (64, 0.1, 1, 1e-11)])
def test_noalloc_fine_batch_equals_fine_batch(torch_cuda, n, eps, prec, tol):
    from paper_1303_6615_amd.binding import Context
    torch = torch_cuda
    nu = NU_BY_NX[n]
    u = np.stack([seeded_state(n, n // 8, 300 + i) for i in range(37)])
    calls = [(u, 0.02, 8), (u[:5], 0.01, 3)]       # the second call: smaller batch, other step size
    print(f"[noalloc] N={n} prec={prec}", flush=True)
    with Context(n, eps, 1.0, nu) as ctx:
        for x, dT, steps in calls:
            xd = torch.tensor(x, device="cuda")
            got = torch.full_like(xd, float("nan"))
            ctx.fine_batch_noalloc(xd, dT, steps, precision=prec, out=got)
            ref = ctx.fine_batch(xd, dT, steps, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (x.shape[0], dT, steps)
            uh = O.project(O.to_spectral(x[:3]), n)
            want = O.to_physical(O.fine_propagate(uh, n, eps, 1.0, nu, dT, steps), n)
            assert _rel(got[:3].cpu().numpy(), want) < tol


def test_noalloc_rejects_a_batch_beyond_its_scratch(torch_cuda):
    from paper_1303_6615_amd.binding import APError, Context
    torch = torch_cuda
    with Context(2048, 0.01, 1.0, 1e-6) as ctx:
        big = torch.zeros((1100, 3, 2048), dtype=torch.float64, device="cuda")
        with pytest.raises(APError, match="exceeds the scratch"):
            ctx.fine_batch_noalloc(big, 0.01, 2, out=torch.empty_like(big))
        ok = ctx.fine_batch_noalloc(big[:1000], 0.01, 2, out=torch.empty_like(big[:1000]))
        torch.cuda.synchronize()
        assert torch.isfinite(ok).all()
