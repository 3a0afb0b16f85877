"""Matrix-core MLP kernels against float64 references.

* the bf16 MFMA GEMM equals a float64 product of the bf16-rounded operands
  (to float32 accumulation error), in all four transposition modes and at
  ragged sizes (several tiles plus a remainder);
* forward and backward of the network match the FP64 oracle MLP to bf16
  tolerances (outputs 2e-2, gradients 5e-2 relative, Frobenius);
* the loss and Adam kernels match their closed forms.
"""
import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _bf16(a):
    return torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (130, 77, 45), (300, 128, 128)])
def test_gemm_bf16_matches_reference(tA, tB, M, N, K):
    from gpu_helpers import need_gpu
    need_gpu()
    from paper_2605_24339_amd.mlp import gemm_bf16
    rng = np.random.default_rng(M * 7 + N + K + tA * 3 + tB)
    A = rng.normal(size=(K, M) if tA else (M, K)).astype(np.float32)
    B = rng.normal(size=(N, K) if tB else (K, N)).astype(np.float32)
    C = gemm_bf16(torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda"), bool(tA), bool(tB))
    Ar, Br = _bf16(A), _bf16(B)
    ref = (Ar.T if tA else Ar) @ (Br.T if tB else Br)
    err = np.abs(C.cpu().numpy() - ref).max()
    assert err <= 1e-5 * np.sqrt(K) * np.abs(ref).max() + 1e-5, err


def test_mlp_forward_backward_match_oracle():
    from gpu_helpers import need_gpu
    need_gpu()
    from paper_2605_24339_amd.mlp import MLP
    rng = np.random.default_rng(5)
    p = omlp.init(2) + rng.normal(size=omlp.N_PARAMS) * 0.01
    B = 1000
    x = np.zeros((B, 16))
    x[:, :9] = rng.normal(size=(B, 9))
    t = np.zeros((B, 16))
    t[:, :3] = rng.normal(size=(B, 3))
    net = MLP(torch.tensor(p, dtype=torch.float32, device="cuda"))
    X = torch.tensor(x, dtype=torch.float32, device="cuda")
    T = torch.tensor(t, dtype=torch.float32, device="cuda")
    y, act = net.forward(X)
    loss, dy = net.mse(y, T)
    g = net.backward(X, act, dy)
    yo, acto = omlp.forward(p, x)
    Lo, dyo = omlp.mse(yo, t)
    go = omlp.backward(p, x, acto, dyo)
    yg = y.double().cpu().numpy()
    assert np.linalg.norm(yg - yo) <= 2e-2 * np.linalg.norm(yo)
    assert abs(loss.item() / Lo - 1) <= 2e-2
    assert np.linalg.norm(g.double().cpu().numpy() - go) <= 5e-2 * np.linalg.norm(go)
    # loss and its gradient on the GPU's own outputs: exact closed form (float32)
    L2, dy2 = omlp.mse(yg, t)
    assert abs(loss.item() / L2 - 1) <= 1e-5
    assert np.abs(dy.double().cpu().numpy() - dy2).max() <= 1e-6 * np.abs(dy2).max()


def test_adam_kernel_matches_closed_form():
    from gpu_helpers import need_gpu
    need_gpu()
    from paper_2605_24339_amd.mlp import MLP
    rng = np.random.default_rng(6)
    p = omlp.init(3)
    net = MLP(torch.tensor(p, dtype=torch.float32, device="cuda"))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    q = p.copy()
    for step in range(1, 4):
        g = rng.normal(size=p.size)
        net.adam(torch.tensor(g, dtype=torch.float32, device="cuda"), lr=1e-2)
        q, m, v = omlp.adam(q, g, m, v, step, lr=1e-2)
    assert np.abs(net.p.double().cpu().numpy() - q).max() <= 1e-5
