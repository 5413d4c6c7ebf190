"""Reference of the surrogate F(lambda) -- TEST INFRASTRUCTURE ONLY.

A 1 -> 64 -> 64 -> 1 tanh network y(t) and its input derivative dy/dt,
trained on value and slope targets with the loss
    L = sum_i wv_i (y_i - yv_i)^2 + ws_i (dy_i - ys_i)^2 .
Parameters (one flat vector): W1[64], b1[64], W2[64][64] (row = output unit),
b2[64], W3[64], b3.

Forward:  a1 = W1 t + b1, h1 = tanh a1, u1 = (1 - h1^2) W1       (u1 = dh1/dt)
          a2 = W2 h1 + b2, h2 = tanh a2, v2 = W2 u1, u2 = (1 - h2^2) v2
          y = W3 . h2 + b3, dy = W3 . u2
Backward: the chain rule through both paths (the slope path needs the
derivative of 1 - h^2, i.e. -2 h).

`bf16=True` rounds exactly where the GPU kernels do: every parameter is used
through its bf16 value; h1, u1, h2, u2 and the layer-2 error signals g_a2,
g_v2 are rounded to bf16 before they enter a product; everything else is
exact (fp64 here, fp32 accumulation on the GPU).  `bf16=False` is the plain
fp64 network, checked against finite differences.
"""
import numpy as np

H = 64
NPARAM = H + H + H * H + H + H + 1


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through fp32, returned as fp64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return rounded.view(np.float32).astype(np.float64)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H]; o += H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1, b1, W2.ravel(), b2, W3, [b3]])


def init_params(seed=0):
    """Glorot-style uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, H) * np.sqrt(6 / (1 + H))
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6 / (2 * H))
    W3 = rng.uniform(-1, 1, H) * np.sqrt(6 / (H + 1))
    return pack(W1, np.zeros(H), W2, np.zeros(H), W3, 0.0)


def forward(theta, t, bf16_round=True):
    r = bf16 if bf16_round else (lambda x: np.asarray(x, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (r(p) for p in unpack(theta))
    t = np.asarray(t, dtype=np.float64)
    a1 = np.outer(t, W1) + b1                 # [n, H]
    h1 = np.tanh(a1)
    u1 = (1.0 - h1 ** 2) * W1
    a2 = r(h1) @ W2.T + b2
    v2 = r(u1) @ W2.T
    h2 = np.tanh(a2)
    u2 = (1.0 - h2 ** 2) * v2
    y = r(h2) @ W3 + b3
    dy = r(u2) @ W3
    return y, dy, dict(t=t, h1=h1, u1=u1, h2=h2, v2=v2, u2=u2)


def loss_and_grad(theta, t, yv, wv, ys, ws, bf16_round=True):
    r = bf16 if bf16_round else (lambda x: np.asarray(x, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (r(p) for p in unpack(theta))
    y, dy, c = forward(theta, t, bf16_round)
    wv = np.asarray(wv, dtype=np.float64); ws = np.asarray(ws, dtype=np.float64)
    ey = 2.0 * wv * (y - yv)
    ed = 2.0 * ws * (dy - ys)
    L = np.sum(wv * (y - yv) ** 2 + ws * (dy - ys) ** 2)
    h1, u1, h2, v2, u2 = c["h1"], c["u1"], c["h2"], c["v2"], c["u2"]
    s1 = 1.0 - h1 ** 2
    s2 = 1.0 - h2 ** 2
    gW3 = ey @ r(h2) + ed @ r(u2)
    gb3 = np.sum(ey)
    g_h2 = np.outer(ey, W3)
    g_u2 = np.outer(ed, W3)
    g_h2 = g_h2 + g_u2 * (-2.0 * h2 * v2)
    g_v2 = g_u2 * s2
    g_a2 = g_h2 * s2
    gb2 = np.sum(g_a2, axis=0)
    ga2r, gv2r = r(g_a2), r(g_v2)
    gW2 = ga2r.T @ r(h1) + gv2r.T @ r(u1)
    g_h1 = ga2r @ W2
    g_u1 = gv2r @ W2
    g_h1 = g_h1 + g_u1 * (-2.0 * h1 * W1)
    gW1 = np.sum(g_u1 * s1, axis=0)
    g_a1 = g_h1 * s1
    gW1 = gW1 + g_a1.T @ c["t"]
    gb1 = np.sum(g_a1, axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(theta, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
