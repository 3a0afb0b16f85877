"""Matrix-core MLP kernels against float64 references.

* the bf16 MFMA GEMM equals a float64 product of the bf16-rounded operands
  (to float32 accumulation error), in all four transposition modes and at
  ragged sizes (several tiles plus a remainder);
* forward and backward of the network match the FP64 oracle MLP to bf16
  tolerances (outputs 2e-2, gradients 5e-2 relative, Frobenius);
* the fused forward equals the layer-by-layer bf16 products (same operand
  rounding, another accumulation order);
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


@pytest.mark.parametrize("B", [1, 31, 1037, 70000])
def test_fused_forward_matches_layer_by_layer_products(B):
    """The fused forward (all layers in one launch, activations in
    registers) against the same network computed layer by layer with the
    bf16 GEMM and float32 bias / SiLU: saved Z and H of every layer and the
    outputs, for batches with a partial last tile of 32 rows and several
    tiles per wave; inference without saved activations gives the same y."""
    from gpu_helpers import need_gpu
    need_gpu()
    from paper_2605_24339_amd.mlp import MLP, gemm_bf16
    rng = np.random.default_rng(B)
    p = omlp.init(3) + rng.normal(size=omlp.N_PARAMS) * 0.01
    x = np.zeros((B, 16), np.float32)
    x[:, :9] = rng.normal(size=(B, 9))
    P = torch.tensor(p, dtype=torch.float32, device="cuda")
    X = torch.tensor(x, device="cuda")
    net = MLP(P)
    y, act = net.forward(X)
    y_inf = torch.empty_like(y)
    from paper_2605_24339_amd.mlp import _lib, _stream
    from paper_2605_24339_amd.gmcp import _ptr
    assert _lib().gmcp_mlp_forward(_ptr(P), _ptr(X), B, _ptr(y_inf), None, _stream(P.device)) == 0
    torch.cuda.synchronize()
    assert torch.equal(y, y_inf)
    o, at = {}, 0
    for name, shp in omlp.SHAPES:
        o[name] = at
        at += int(np.prod(shp))
    W = lambda k, r, c: P[o[k]:o[k] + r * c].reshape(r, c)
    b = lambda k, n: P[o[k]:o[k] + n]
    silu = lambda z: z * torch.sigmoid(z)
    h, zs, hs = X, [], []
    for k in (1, 2, 3):
        fin = 16 if k == 1 else 128
        z = gemm_bf16(h, W(f"W{k}", fin, 128).contiguous()) + b(f"b{k}", 128)
        h = silu(z)
        zs.append(z)
        hs.append(h)
    yr = gemm_bf16(h, W("W4", 128, 16).contiguous()) + b("b4", 16)
    rel = lambda a, r: float((a - r).norm() / r.norm())
    for k in range(3):
        assert rel(act[:, 256 * k:256 * k + 128], zs[k]) <= 2e-3, k
        assert rel(act[:, 256 * k + 128:256 * k + 256], hs[k]) <= 2e-3, k
    assert rel(y, yr) <= 2e-3


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
