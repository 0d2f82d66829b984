"""Plain FP64 reference of the learned smoother (test infrastructure only).

The network (no counterpart in the paper; the learned-smoother extension of the
multigrid V-cycle of Sec. 4.1 / Example 4.3):

  input  x0 (8 channels per lattice site): the residual r scaled by its RMS s
         (Re r_0, Im r_0, Re r_1, Im r_1 for the two spins), then cos and sin of
         the link phases theta_0 and theta_1 at the site;
  layer 1: 3x3 convolution 8 -> 16 channels, ReLU;
  layer 2: 3x3 convolution 16 -> 16 channels, ReLU;
  layer 3: 3x3 convolution 16 -> 4 channels (linear);
  output: the correction e = s * (o_0 + i o_1, o_2 + i o_3) per site.

Convolutions are cross-correlations without bias,
  y[co, i, j] = sum_{ci, a, b} W[co, ci, a, b] * x[ci, i + a - 1, j + b - 1],
periodic on the N x N lattice; on training crops they are "valid" (no padding,
each layer shrinks the crop by 2).  Training loss: mean squared error over the
output sites and channels.  Weights: W1 [16, 8, 3, 3], W2 [16, 16, 3, 3],
W3 [4, 16, 3, 3]; flattened in that order (4032 values).
"""
import numpy as np

SHAPES = ((16, 8, 3, 3), (16, 16, 3, 3), (4, 16, 3, 3))
N_WEIGHTS = sum(int(np.prod(s)) for s in SHAPES)


def unflatten(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_WEIGHTS
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(w[o:o + k].reshape(s))
        o += k
    return out


def flatten(Ws):
    return np.concatenate([np.asarray(W, dtype=np.float64).ravel() for W in Ws])


def conv3x3(x, W, periodic):
    """x [Ci, H, W_] -> [Co, H, W_] (periodic) or [Co, H-2, W_-2] (valid)."""
    x = np.asarray(x, dtype=np.float64)
    Co = W.shape[0]
    if periodic:
        H, Wd = x.shape[1:]
        y = np.zeros((Co, H, Wd))
        for a in range(3):
            for b in range(3):
                # shifted[ci, i, j] = x[ci, i + a - 1, j + b - 1]
                shifted = np.roll(x, shift=(1 - a, 1 - b), axis=(1, 2))
                y += np.einsum("oc,chw->ohw", W[:, :, a, b], shifted)
        return y
    H, Wd = x.shape[1] - 2, x.shape[2] - 2
    y = np.zeros((Co, H, Wd))
    for a in range(3):
        for b in range(3):
            y += np.einsum("oc,chw->ohw", W[:, :, a, b], x[:, a:a + H, b:b + Wd])
    return y


def forward(x0, Ws, periodic):
    """Activations (pre-activation z, post-activation h) of every layer."""
    z1 = conv3x3(x0, Ws[0], periodic)
    h1 = np.maximum(z1, 0.0)
    z2 = conv3x3(h1, Ws[1], periodic)
    h2 = np.maximum(z2, 0.0)
    out = conv3x3(h2, Ws[2], periodic)
    return dict(x0=x0, z1=z1, h1=h1, z2=z2, h2=h2, out=out)


def features(r, theta, N):
    """(x0 [8, N, N], s) from the residual r (2 N^2 complex, spin innermost,
    site y*N + x) and the link phases theta [2, N, N]."""
    r = np.asarray(r, dtype=np.complex128).reshape(N, N, 2)
    s = np.sqrt(np.mean(np.abs(r) ** 2))
    rh = r / s if s > 0 else r
    x0 = np.stack([rh[..., 0].real, rh[..., 0].imag, rh[..., 1].real, rh[..., 1].imag,
                   np.cos(theta[0]), np.sin(theta[0]), np.cos(theta[1]), np.sin(theta[1])])
    return x0, s


def correction(r, theta, N, w):
    """The smoother's correction e (2 N^2 complex) for the residual r."""
    x0, s = features(r, theta, N)
    o = forward(x0, unflatten(w), periodic=True)["out"]
    e = np.empty((N, N, 2), dtype=np.complex128)
    e[..., 0] = s * (o[0] + 1j * o[1])
    e[..., 1] = s * (o[2] + 1j * o[3])
    return e.reshape(-1)


def _conv_grads(x, W, dy):
    """For y = conv3x3(x, W, valid): dL/dW and dL/dx given dL/dy."""
    Ho, Wo = dy.shape[1:]
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    for a in range(3):
        for b in range(3):
            xs = x[:, a:a + Ho, b:b + Wo]
            dW[:, :, a, b] = np.einsum("ohw,chw->oc", dy, xs)
            dx[:, a:a + Ho, b:b + Wo] += np.einsum("oc,ohw->chw", W[:, :, a, b], dy)
    return dW, dx


def loss_and_grad(X0, T, w):
    """Mean squared error of the valid-convolution network on crops and its
    gradient with respect to the flattened weights.

    X0: [B, 8, H, W] inputs; T: [B, 4, H-6, W-6] targets."""
    Ws = unflatten(w)
    X0 = np.asarray(X0, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    count = T.size
    loss = 0.0
    g = [np.zeros_like(W) for W in Ws]
    for x0, t in zip(X0, T):
        act = forward(x0, Ws, periodic=False)
        d = act["out"] - t
        loss += np.sum(d * d)
        dout = 2.0 * d / count
        dW3, dh2 = _conv_grads(act["h2"], Ws[2], dout)
        dz2 = dh2 * (act["z2"] > 0)
        dW2, dh1 = _conv_grads(act["h1"], Ws[1], dz2)
        dz1 = dh1 * (act["z1"] > 0)
        dW1, _ = _conv_grads(act["x0"], Ws[0], dz1)
        g[0] += dW1
        g[1] += dW2
        g[2] += dW3
    return loss / count, flatten(g)


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, bias-corrected); t counts from 1.
    Returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
