"""gmcp_mlp_mse_noalloc: the mean-squared loss and its gradient with the
partial sums in the library's static device scratch instead of a caller
workspace (for callers that cannot allocate).  Through the C ABI, two calls
in a row (the second on fewer rows, so it reads only partials it wrote
itself) must equal gmcp_mlp_mse with a workspace bit for bit, and the loss
must match a float64 reference; a batch beyond the scratch is rejected
before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import need_gpu

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _p(t):
    return C.c_void_p(t.data_ptr())


def _with_work(L, y, t, n_out, stream):
    B = y.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    nbytes = 4 * ((B * 16 + 255) // 256 + 1)
    work = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    assert L.gmcp_mlp_mse(_p(y), _p(t), B, n_out, _p(loss), _p(dy), _p(work), nbytes, stream) == 0
    return loss, dy


def _no_alloc(L, y, t, n_out, stream):
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    dy = torch.full_like(y, float("nan"))
    assert L.gmcp_mlp_mse_noalloc(_p(y), _p(t), y.shape[0], n_out, _p(loss), _p(dy), stream) == 0
    return loss, dy


def test_no_alloc_mse_matches_workspace_version():
    need_gpu()
    from paper_2605_24339_amd import _native as N
    from paper_2605_24339_amd.mlp import _lib
    L = _lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cpu").manual_seed(5)
    for B, n_out in ((300_001, 3), (1_000, 16)):       # second call: fewer rows
        y = torch.randn(B, 16, generator=g).cuda()
        t = torch.randn(B, 16, generator=g).cuda()
        l0, d0 = _with_work(L, y, t, n_out, stream)
        l1, d1 = _no_alloc(L, y, t, n_out, stream)
        torch.cuda.synchronize()
        assert torch.equal(l0, l1), (B, l0.item(), l1.item())
        assert torch.equal(d0, d1), B
        yd, td = y.double().cpu().numpy(), t.double().cpu().numpy()
        diff = yd[:, :n_out] - td[:, :n_out]
        ref = float((diff ** 2).mean())
        assert abs(l1.item() / ref - 1) <= 1e-5
        assert np.allclose(d1.double().cpu().numpy()[:, :n_out], 2 * diff / (B * n_out), rtol=1e-6, atol=0)
        assert torch.all(d1[:, n_out:] == 0)
    big = int(L.gmcp_mlp_mse_noalloc_max_rows()) + 1
    x = torch.zeros(1, 16, device="cuda")
    assert L.gmcp_mlp_mse_noalloc(_p(x), _p(x), big, 3, _p(x), _p(x), stream) == N.GMCP_E_ARG
