"""GPU checks of the warm-start network kernels against the float64 oracle.

Bars: the BF16 MFMA GEMM against a float64 product of the same bf16-rounded
operands (float32 accumulation: 1e-5 relative); every layer shape of the
network run alone (forward output, input gradient, weight and bias
gradients) on operands that bfloat16 represents exactly, so that only the
float32 accumulation differs from oracle/cnn.py: 1e-5 relative (L2 and
largest entry); the whole network's forward output, loss and parameter
gradient (bfloat16 rounding of the activations and gradients between layers
carries ~2^-8 relative error through six layers: 3e-2 relative L2 on the
output and the gradient, 1e-2 on the loss); features, scaling and Adam in
float32 against float64 (1e-6).
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


def _bf16_exact(rng, shape, scale=1.0):
    """Random values that bfloat16 represents exactly (float64 array)."""
    a = torch.as_tensor(scale * rng.standard_normal(shape), dtype=torch.float32)
    return a.to(torch.bfloat16).to(torch.float64).numpy()


# (batch, Hi, Wi, cin, cout, stride, up, Hs, Ws): the six layer shapes of the
# network for N_f = 2 and 3 on a 17 x 19 grid (layers 4 and 5 read the nearest
# x2 up-sampling of their input, cut to the window grid Hs x Ws)
CONV_CASES = [
    (2, 17, 19, 12, 32, 1, 0, 17, 19),
    (2, 17, 19, 32, 64, 2, 0, 17, 19),
    (2, 9, 10, 64, 64, 2, 0, 9, 10),
    (2, 5, 5, 64, 64, 1, 1, 9, 10),
    (2, 9, 10, 64, 32, 1, 1, 17, 19),
    (2, 17, 19, 32, 3, 1, 0, 17, 19),
    (1, 40, 33, 18, 32, 1, 0, 40, 33),
]


@pytest.mark.parametrize("case", CONV_CASES, ids=lambda c: "x".join(map(str, c)))
def test_cnn_single_layer_forward_backward_bf16_exact(case):
    """One 3x3 convolution layer through the C ABI (the im2col, BF16 MFMA
    GEMM, bias, col2im, weight-unpacking and up-sampling kernels the network
    chains) against oracle/cnn.py's conv / conv_backward / up2 on operands
    exact in bfloat16: relative L2 and largest-entry error <= 1e-5 for z,
    dx, dW and db."""
    L = _L()
    B, Hi, Wi, ci, co, st, up, Hs, Ws = case
    rng = np.random.default_rng(sum(case))
    x = _bf16_exact(rng, (B, ci, Hi, Wi))
    Wt = _bf16_exact(rng, (co, ci, 3, 3), 0.2)
    b = _bf16_exact(rng, (co,), 0.5)
    u = cnn.up2(x, Hs, Ws) if up else x
    z_ref = cnn.conv(u, Wt, b, st)
    dz = _bf16_exact(rng, z_ref.shape)
    du, dW_ref, db_ref = cnn.conv_backward(u, Wt, dz, st)
    dx_ref = cnn.up2_backward(du, Hi, Wi) if up else du
    nbytes = L.mfwh_cnn_conv3x3_workspace_bytes(B, Hi, Wi, ci, co, st, up, Hs, Ws)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    wb = torch.as_tensor(np.concatenate([Wt.ravel(), b]), dtype=torch.float32, device="cuda")
    xd = _to_gpu_nhwc(x)
    Ho, Wo = z_ref.shape[2], z_ref.shape[3]
    z = torch.empty((B, Ho, Wo, co), dtype=torch.float32, device="cuda")
    L.mfwh_cnn_conv3x3(B, Hi, Wi, ci, co, st, up, Hs, Ws, xd, wb, z, None, None, None, ws)
    dx = torch.empty_like(xd)
    dwb = torch.empty_like(wb)
    L.mfwh_cnn_conv3x3(B, Hi, Wi, ci, co, st, up, Hs, Ws, xd, wb, None, _to_gpu_nhwc(dz), dx,
                       dwb, ws)
    torch.cuda.synchronize()
    got = dict(z=z.cpu().double().numpy().transpose(0, 3, 1, 2),
               dx=dx.cpu().double().numpy().transpose(0, 3, 1, 2),
               dW=dwb.cpu().double().numpy()[:co * ci * 9].reshape(co, ci, 3, 3),
               db=dwb.cpu().double().numpy()[co * ci * 9:])
    ref = dict(z=z_ref, dx=dx_ref, dW=dW_ref, db=db_ref)
    for k in ref:
        e2 = rel(got[k], ref[k])
        emax = float(np.max(np.abs(got[k] - ref[k])) / np.max(np.abs(ref[k])))
        assert e2 < 1e-5 and emax < 1e-5, (k, e2, emax)


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
