"""GPU checks of the warm-start network kernels against the float64 oracle.

Bars: the BF16 MFMA GEMM against a float64 product of the same bf16-rounded
operands (float32 accumulation: 1e-5 relative); the network forward output,
loss and parameter gradient against oracle/cnn.py (bfloat16 operands carry
~2^-8 relative rounding through six layers: 3e-2 relative L2 on the output and
the whole gradient, 1e-2 on the loss, 0.15 per layer); features, scaling and
Adam in float32 against float64 (1e-6).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cnn  # noqa: E402


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _L():
    from paper_2507_23613_amd import _lib
    return _lib


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("atrans", [0, 1])
@pytest.mark.parametrize("M,N,K", [(16, 16, 16), (70, 33, 50), (257, 64, 576), (300, 40, 20000)])
def test_gemm_bf16_matches_float64(atrans, M, N, K):
    L = _L()
    g = torch.Generator(device="cpu").manual_seed(M * 7 + N + K)
    A = torch.randn(M, K, generator=g).to(torch.bfloat16)
    B = torch.randn(K, N, generator=g).to(torch.bfloat16)
    ref = A.double().numpy() @ B.double().numpy()
    Ad = (A.t().contiguous() if atrans else A).cuda()
    Bd = B.contiguous().cuda()
    C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
    part = torch.empty(64 * M * N, dtype=torch.float32, device="cuda")
    lda = M if atrans else K
    L.mfwh_gemm_bf16(Ad.view(torch.int16), Bd.view(torch.int16), C, atrans, M, N, K, lda, N, N,
                     part)
    torch.cuda.synchronize()
    assert rel(C.cpu().double().numpy(), ref) < 1e-5


def _net_case(B=2, nf=2, H=17, W=19, seed=0):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(nf, seed=seed) * 0.7
    p += 0.05 * rng.standard_normal(p.size)
    x = rng.standard_normal((B, 6 * nf, H, W))
    t = rng.standard_normal((B, nf, H, W))
    return p, x, t


def _to_gpu_nhwc(a):
    return torch.as_tensor(np.ascontiguousarray(a.transpose(0, 2, 3, 1)), dtype=torch.float32,
                           device="cuda")


@pytest.mark.parametrize("shape", [(2, 2, 17, 19), (1, 4, 32, 32), (3, 1, 9, 12)])
def test_cnn_forward_matches_oracle(shape):
    L = _L()
    B, nf, H, W = shape
    p, x, _ = _net_case(B, nf, H, W)
    ref = cnn.forward(p, x, nf)
    ws = torch.empty(L.mfwh_cnn_workspace_bytes(B, nf, H, W), dtype=torch.uint8, device="cuda")
    out = torch.empty((B, H, W, nf), dtype=torch.float32, device="cuda")
    L.mfwh_cnn_forward(torch.as_tensor(p, dtype=torch.float32, device="cuda"), _to_gpu_nhwc(x),
                       out, nf, ws)
    torch.cuda.synchronize()
    got = out.cpu().double().numpy().transpose(0, 3, 1, 2)
    assert rel(got, ref) < 3e-2


@pytest.mark.parametrize("shape", [(2, 2, 17, 19), (1, 3, 24, 20)])
def test_cnn_loss_and_gradient_match_oracle(shape):
    L = _L()
    B, nf, H, W = shape
    p, x, t = _net_case(B, nf, H, W, seed=1)
    loss_ref, g_ref = cnn.loss_and_grad(p, x, t, nf)
    ws = torch.empty(L.mfwh_cnn_workspace_bytes(B, nf, H, W), dtype=torch.uint8, device="cuda")
    grad = torch.empty(p.size, dtype=torch.float32, device="cuda")
    loss = L.mfwh_cnn_loss_grad(torch.as_tensor(p, dtype=torch.float32, device="cuda"),
                                _to_gpu_nhwc(x), _to_gpu_nhwc(t), grad, nf, ws)
    g = grad.cpu().double().numpy()
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    assert rel(g, g_ref) < 3e-2
    # per layer too (each block of the flat vector); a layer's weight gradient
    # is a sum over all pixels of bf16 products that can cancel strongly
    # (measured up to 0.11 for the first layer), hence the looser bar
    o = 0
    for co, ci in cnn.layer_shapes(nf):
        nw = co * ci * 9
        assert rel(g[o:o + nw], g_ref[o:o + nw]) < 0.15
        o += nw + co


def test_cnn_features_and_scale_match_oracle():
    L = _L()
    rng = np.random.default_rng(3)
    B, nf, H, W = 2, 3, 11, 13
    f = rng.standard_normal((B, nf, H, W))
    omega = rng.uniform(5, 40, (B, nf))
    ws = torch.empty(L.mfwh_cnn_workspace_bytes(B, nf, H, W), dtype=torch.uint8, device="cuda")
    fd = torch.as_tensor(f, device="cuda")
    od = torch.as_tensor(omega, device="cuda")
    feat = torch.empty((B, H, W, 6 * nf), dtype=torch.float32, device="cuda")
    L.mfwh_cnn_features(fd, od, (1.0, 1.3), feat, ws)
    for b in range(B):
        ref = cnn.features(f[b], omega[b], lengths=(1.0, 1.3))
        got = feat[b].cpu().double().numpy().transpose(2, 0, 1)
        assert np.allclose(got, ref, atol=2e-6)
    # dir 1 (targets) then dir 0 (back to fields) round trip, against the scale
    v = torch.as_tensor(rng.standard_normal((B, nf, H, W)), device="cuda")
    out = torch.empty((B, H, W, nf), dtype=torch.float32, device="cuda")
    L.mfwh_cnn_scale(1, out, v, fd, od, ws)
    v2 = torch.empty_like(v)
    L.mfwh_cnn_scale(0, out, v2, fd, od, ws)
    for b in range(B):
        s = cnn.target_scale(f[b], omega[b])
        o = out[b].cpu().double().numpy().transpose(2, 0, 1)
        assert np.allclose(o * s[:, None, None], v[b].cpu().numpy(), rtol=1e-6, atol=1e-9)
        inner = v2[b].cpu().numpy()[:, 1:-1, 1:-1]
        assert np.allclose(inner, v[b].cpu().numpy()[:, 1:-1, 1:-1], rtol=1e-6, atol=1e-9)
        assert np.all(v2[b].cpu().numpy()[:, 0, :] == 0)


def test_cnn_adam_matches_oracle():
    L = _L()
    rng = np.random.default_rng(4)
    p, g = rng.standard_normal(1000), rng.standard_normal(1000)
    m, v = 0.1 * rng.standard_normal(1000), np.abs(rng.standard_normal(1000))
    pd, gd, md, vd = (torch.as_tensor(a, dtype=torch.float32, device="cuda") for a in (p, g, m, v))
    L.mfwh_cnn_adam(pd, gd, md, vd, 3, 1e-3)
    p1, m1, v1 = cnn.adam(p, g, m, v, 3, 1e-3)
    assert np.allclose(pd.cpu().numpy(), p1, rtol=1e-6, atol=1e-7)
    assert np.allclose(md.cpu().numpy(), m1, rtol=1e-6, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), v1, rtol=1e-6, atol=1e-7)


def test_cnn_training_reduces_loss():
    """A few Adam steps on one batch lower the loss (kernels compose)."""
    L = _L()
    B, nf, H, W = 2, 2, 32, 32
    p, x, t = _net_case(B, nf, H, W, seed=5)
    ws = torch.empty(L.mfwh_cnn_workspace_bytes(B, nf, H, W), dtype=torch.uint8, device="cuda")
    pd = torch.as_tensor(p, dtype=torch.float32, device="cuda")
    m, v = torch.zeros_like(pd), torch.zeros_like(pd)
    g = torch.empty_like(pd)
    xd, td = _to_gpu_nhwc(x), _to_gpu_nhwc(0.1 * t)
    losses = []
    for step in range(1, 31):
        losses.append(L.mfwh_cnn_loss_grad(pd, xd, td, g, nf, ws))
        L.mfwh_cnn_adam(pd, g, m, v, step, 3e-3)
    assert losses[-1] < 0.5 * losses[0]
