"""Plain FP64 forward/backward of the warm-start network (oracle; test infrastructure only).

Test infrastructure only: nothing in the product imports this module.

The network is not part of the paper: it is the learned start vector of the
pressure Poisson solve.  Four 3x3 convolution layers on a lattice image
(channels: scaled residual of the previous pressure increment, scaled
right-hand side, lattice mask), 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first
three, zero padding.  Its output is the scaled change of the increment.

Conventions shared with the HIP kernels by specification:
* images are NHWC, y[b,i,j,co] = bias[co] + sum_{ky,kx,ci} x[b,i+ky-1,j+kx-1,ci] W[ky,kx,ci,co]
  (cross-correlation; values outside the image are zero);
* flat parameter vector: W1 [3,3,3,32], b1 [32], W2 [3,3,32,32], b2, W3 [3,3,32,32], b3,
  W4 [3,3,32,1], b4 [1];
* loss: masked mean squared error sum(m (y - t)^2) / sum(m);
* Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Each convolution is a sum over the nine taps of a channel matmul (numpy
matmul is the library step), written with no blocking or fusion.
"""
import numpy as np

SHAPES = [(3, 3, 3, 32), (32,), (3, 3, 32, 32), (32,), (3, 3, 32, 32), (32,), (3, 3, 32, 1), (1,)]


def n_params():
    return int(sum(np.prod(s) for s in SHAPES))


def unflatten(theta):
    out, k = [], 0
    for s in SHAPES:
        m = int(np.prod(s))
        out.append(np.asarray(theta[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed):
    """He-uniform weights, zero biases (used only to make test inputs)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 4:
            fan_in = s[0] * s[1] * s[2]
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, s))
        else:
            parts.append(np.zeros(s))
    return flatten(parts)


def _shift(x, dy, dx):
    """out[b,i,j] = x[b,i+dy,j+dx] with zeros outside."""
    out = np.zeros_like(x)
    H, W = x.shape[1], x.shape[2]
    i0, i1 = max(0, -dy), min(H, H - dy)
    j0, j1 = max(0, -dx), min(W, W - dx)
    out[:, i0:i1, j0:j1] = x[:, i0 + dy:i1 + dy, j0 + dx:j1 + dx]
    return out


def conv(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[3],))
    for ky in range(3):
        for kx in range(3):
            y += _shift(x, ky - 1, kx - 1) @ W[ky, kx]
    return y + b


def conv_backward(x, W, gy):
    """Gradients of sum(gy * conv(x, W, b)) with respect to x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            xs = _shift(x, ky - 1, kx - 1)
            gW[ky, kx] = np.einsum("bijc,bijo->co", xs, gy)
            gx += _shift(gy @ W[ky, kx].T, -(ky - 1), -(kx - 1))
    return gx, gW, gy.sum(axis=(0, 1, 2))


def forward(theta, x):
    """Returns the prediction [B,H,W] and the list of layer inputs (for backward)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(theta)
    a0 = np.asarray(x, dtype=np.float64)
    a1 = np.maximum(conv(a0, W1, b1), 0.0)
    a2 = np.maximum(conv(a1, W2, b2), 0.0)
    a3 = np.maximum(conv(a2, W3, b3), 0.0)
    y = conv(a3, W4, b4)[..., 0]
    return y, [a0, a1, a2, a3]


def loss_and_grad(theta, x, target, mask):
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(theta)
    y, (a0, a1, a2, a3) = forward(theta, x)
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum()
    diff = y - target
    loss = float((m * diff * diff).sum() / cnt)
    g = (2.0 * m * diff / cnt)[..., None]
    g3, gW4, gb4 = conv_backward(a3, W4, g)
    g3 = g3 * (a3 > 0)
    g2, gW3, gb3 = conv_backward(a2, W3, g3)
    g2 = g2 * (a2 > 0)
    g1, gW2, gb2 = conv_backward(a1, W2, g2)
    g1 = g1 * (a1 > 0)
    _, gW1, gb1 = conv_backward(a0, W1, g1)
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
