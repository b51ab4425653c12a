"""Oracle: the warm-start convolutional network in float64 (forward, backward,
Adam), written plainly with NumPy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The network is not
part of the paper (the learned warm start is an addition to the method); its
definition here is the reference the GPU kernels are checked against, and
this module is pinned by finite differences and closed-form special cases.

Network (NCHW, 3x3 convolutions with zero padding 1, bias):
  a1 = relu(conv(x, W1))                     C0 -> 32, stride 1
  a2 = relu(conv(a1, W2, stride 2))          32 -> 64
  a3 = relu(conv(a2, W3, stride 2))          64 -> 64
  a4 = relu(conv(up2(a3), W4)) + a2          64 -> 64   (up2: nearest x2)
  a5 = relu(conv(up2(a4), W5)) + a1          64 -> 32
  y  = conv(a5, W6)                          32 -> nf
Parameters are one flat float vector: for each layer W (cout, cin, 3, 3)
then b (cout).  Loss: mean of (y - target)^2 over every element.
"""
import numpy as np

C1, C2 = 32, 64


def layer_shapes(nf, c0=None):
    c0 = 6 * nf if c0 is None else c0
    return [(C1, c0), (C2, C1), (C2, C2), (C2, C2), (C1, C2), (nf, C1)]


def param_count(nf, c0=None):
    return sum(co * ci * 9 + co for co, ci in layer_shapes(nf, c0))


def unpack(p, nf, c0=None):
    out, o = [], 0
    for co, ci in layer_shapes(nf, c0):
        W = p[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = p[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(nf, seed=0, c0=None):
    """He-normal weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in layer_shapes(nf, c0):
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def conv(x, W, b, stride=1):
    """x (B, ci, H, W) -> (B, co, Ho, Wo); out[y,x] = sum W[co,ci,ky,kx] *
    xpad[ci, s*y + ky, s*x + kx] + b[co] (padding 1)."""
    B, ci, H, Wd = x.shape
    Ho, Wo = (H - 1) // stride + 1, (Wd - 1) // stride + 1
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((B, W.shape[0], Ho, Wo))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += np.einsum("oc,bchw->bohw", W[:, :, ky, kx], patch)
    return out + b[None, :, None, None]


def conv_backward(x, W, dout, stride=1):
    """Gradients of conv w.r.t. x, W, b given dout."""
    B, ci, H, Wd = x.shape
    Ho, Wo = dout.shape[2], dout.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dout, xp[sl])
            dxp[sl] += np.einsum("oc,bohw->bchw", W[:, :, ky, kx], dout)
    db = dout.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dW, db


def up2(x, H, W):
    """Nearest-neighbour upsampling to (H, W): out[y, x] = in[y // 2, x // 2]."""
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)[:, :, :H, :W]


def up2_backward(d, h, w):
    out = np.zeros(d.shape[:2] + (h, w))
    H, W = d.shape[2], d.shape[3]
    for dy in range(2):
        for dx in range(2):
            part = d[:, :, dy::2, dx::2]
            out[:, :, :part.shape[2], :part.shape[3]] += part
    return out


def forward(p, x, nf, keep=False):
    (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5), (W6, b6) = unpack(p, nf, x.shape[1])
    H, Wd = x.shape[2], x.shape[3]
    z1 = conv(x, W1, b1)
    a1 = np.maximum(z1, 0)
    z2 = conv(a1, W2, b2, 2)
    a2 = np.maximum(z2, 0)
    z3 = conv(a2, W3, b3, 2)
    a3 = np.maximum(z3, 0)
    u3 = up2(a3, a2.shape[2], a2.shape[3])
    z4 = conv(u3, W4, b4)
    a4 = np.maximum(z4, 0) + a2
    u4 = up2(a4, H, Wd)
    z5 = conv(u4, W5, b5)
    a5 = np.maximum(z5, 0) + a1
    y = conv(a5, W6, b6)
    if keep:
        return y, dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, u3=u3, z4=z4, a4=a4,
                       u4=u4, z5=z5, a5=a5)
    return y


def loss_and_grad(p, x, target, nf):
    """Mean-squared-error loss and its gradient w.r.t. the flat parameters."""
    y, c = forward(p, x, nf, keep=True)
    (W1, _), (W2, _), (W3, _), (W4, _), (W5, _), (W6, _) = unpack(p, nf, x.shape[1])
    diff = y - target
    loss = float(np.mean(diff ** 2))
    dy = 2.0 * diff / diff.size
    da5, dW6, db6 = conv_backward(c["a5"], W6, dy)
    dz5 = da5 * (c["z5"] > 0)
    da1_skip = da5
    du4, dW5, db5 = conv_backward(c["u4"], W5, dz5)
    da4 = up2_backward(du4, c["a4"].shape[2], c["a4"].shape[3])
    dz4 = da4 * (c["z4"] > 0)
    da2_skip = da4
    du3, dW4, db4 = conv_backward(c["u3"], W4, dz4)
    da3 = up2_backward(du3, c["a3"].shape[2], c["a3"].shape[3])
    dz3 = da3 * (c["z3"] > 0)
    da2, dW3, db3 = conv_backward(c["a2"], W3, dz3, 2)
    da2 = da2 + da2_skip
    dz2 = da2 * (c["z2"] > 0)
    da1, dW2, db2 = conv_backward(c["a1"], W2, dz2, 2)
    da1 = da1 + da1_skip
    dz1 = da1 * (c["z1"] > 0)
    _, dW1, db1 = conv_backward(c["x"], W1, dz1)
    g = np.concatenate([t.ravel() for t in (dW1, db1, dW2, db2, dW3, db3, dW4, db4, dW5, db5,
                                             dW6, db6)])
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); returns new (p, m, v).  step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(f, omega, lengths=(1.0, 1.0)):
    """Input channels of one problem (nf, H, W) full grid with boundary:
    f_m / max|f_m|, sin(omega_m x), cos(omega_m x), sin(omega_m y),
    cos(omega_m y), omega_m / 50 (constant); 6 nf channels."""
    nf, H, W = f.shape
    y = np.linspace(0, lengths[0], H)[:, None] * np.ones((1, W))
    x = np.ones((H, 1)) * np.linspace(0, lengths[1], W)[None, :]
    ch = []
    for m in range(nf):
        s = np.max(np.abs(f[m]))
        ch.append(f[m] / s if s > 0 else f[m])
    for m in range(nf):
        ch.append(np.sin(omega[m] * x))
    for m in range(nf):
        ch.append(np.cos(omega[m] * x))
    for m in range(nf):
        ch.append(np.sin(omega[m] * y))
    for m in range(nf):
        ch.append(np.cos(omega[m] * y))
    for m in range(nf):
        ch.append(np.full((H, W), omega[m] / 50.0))
    return np.stack(ch)


def target_scale(f, omega):
    """Scale between the network output and the solution:
    U_m = out_m * max|f_m| / omega_m^2."""
    return np.array([np.max(np.abs(f[m])) / omega[m] ** 2 for m in range(f.shape[0])])
