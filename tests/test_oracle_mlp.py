"""Pins of the surrogate reference (oracle/mlp.py) -- no GPU."""
import numpy as np

from oracle import mlp


def _data(n=37, seed=1):
    rng = np.random.default_rng(seed)
    t = rng.uniform(-1, 1, n)
    return t, np.sin(2 * t), rng.uniform(0.5, 1.5, n), 2 * np.cos(2 * t), rng.uniform(0.1, 0.9, n)


def test_gradient_matches_finite_differences():
    th = mlp.init_params(3)
    th[mlp.H:2 * mlp.H] = 0.1          # non-zero biases so every path is exercised
    t, yv, wv, ys, ws = _data()
    L, g = mlp.loss_and_grad(th, t, yv, wv, ys, ws, bf16_round=False)
    rng = np.random.default_rng(0)
    idx = np.concatenate([np.arange(5), mlp.H + np.arange(3), 2 * mlp.H + rng.integers(0, 4096, 20),
                          mlp.NPARAM - 66 + np.arange(3), [mlp.NPARAM - 1]])
    for i in idx:
        e = np.zeros_like(th); e[i] = 1e-6
        fd = (mlp.loss_and_grad(th + e, t, yv, wv, ys, ws, False)[0] -
              mlp.loss_and_grad(th - e, t, yv, wv, ys, ws, False)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_slope_output_is_input_derivative():
    th = mlp.init_params(5)
    t = np.linspace(-1, 1, 11)
    y, dy, _ = mlp.forward(th, t, bf16_round=False)
    h = 1e-6
    fd = (mlp.forward(th, t + h, False)[0] - mlp.forward(th, t - h, False)[0]) / (2 * h)
    assert np.allclose(dy, fd, atol=1e-8)


def test_special_cases():
    # zero weights: y = b3, dy = 0; tanh'(0) = 1 so with W2 = I, b = 0: dy(0) = W3 . W1
    W1 = np.linspace(-1, 1, mlp.H); W3 = np.linspace(0.5, -0.5, mlp.H)
    th = mlp.pack(W1, np.zeros(mlp.H), np.eye(mlp.H), np.zeros(mlp.H), W3, 0.25)
    y, dy, _ = mlp.forward(th, np.array([0.0]), bf16_round=False)
    assert y[0] == 0.25 and abs(dy[0] - W3 @ W1) < 1e-14
    z = mlp.pack(np.zeros(mlp.H), np.zeros(mlp.H), np.zeros((mlp.H, mlp.H)), np.zeros(mlp.H), np.zeros(mlp.H), -3.0)
    y, dy, _ = mlp.forward(z, np.linspace(-1, 1, 5))
    assert np.all(y == -3.0) and np.all(dy == 0.0)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 1e-3])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                                            # 1 + 2^-8 is a tie -> even (1.0)
    assert r[2] == 1.0 + 2 ** -7                                  # above the tie -> up
    assert r[3] == -2.5
    assert abs(r[4] - 1e-3) <= 2 ** -9 * 1e-3


def test_adam_reduces_loss_and_fits_a_line():
    """Least squares with value targets on y = 0.3 t - 0.2 through the network: Adam
    drives the loss down by orders of magnitude (a textbook linear fit reached through
    the nonlinear model)."""
    th = mlp.init_params(7)
    t = np.linspace(-1, 1, 64)
    yv = 0.3 * t - 0.2
    wv = np.ones_like(t); ws = np.zeros_like(t)
    m = np.zeros_like(th); v = np.zeros_like(th)
    L0 = mlp.loss_and_grad(th, t, yv, wv, yv, ws, False)[0]
    for k in range(1, 400):
        L, g = mlp.loss_and_grad(th, t, yv, wv, yv, ws, False)
        th, m, v = mlp.adam(th, g, m, v, 3e-3, k)
    assert L < 1e-3 * L0


def test_adam_closed_form_steps():
    """Adam's update written out by hand (Kingma & Ba, beta1 = 0.9, beta2 = 0.999,
    eps = 1e-8 outside the square root, bias correction by 1 - beta^t):
      * step 1: m^ = g and v^ = g^2 exactly, so every parameter moves by
        -lr g / (|g| + eps): lr against the sign of g for |g| >> eps, and
        lr/11 for |g| = eps/10 (eps inside the root would give lr 1e-5 there;
        no bias correction would give lr sqrt(1000)/10 = 3.16 lr);
      * a constant gradient keeps m^ = g and v^ = g^2 at every step, so every
        step moves by the same -lr g / (|g| + eps) (a wrong power of beta in
        the correction breaks this from step 2 on);
      * g = 2 then g = -1: m_2 = 0.9*0.1*2 - 0.1 = 0.08, m^_2 = 0.08/0.19;
        v_2 = 0.999*0.001*4 + 0.001 = 0.004996, v^_2 = 0.004996/0.001999."""
    lr = 1e-3
    g = np.array([2.0, -0.5, 1e-9, -3e4])
    th1, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), lr, 1)
    assert np.allclose(th1[[0, 1, 3]], [-lr, lr, lr], rtol=1e-7, atol=0)
    assert abs(th1[2] - (-lr / 11.0)) < 1e-12 * lr
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-15)
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    gc = np.array([0.7, -2.0, 5.0, -1e-3])
    for step in range(1, 8):
        prev = th.copy()
        th, m, v = mlp.adam(th, gc, m, v, lr, step)
        assert np.allclose(th - prev, -lr * gc / (np.abs(gc) + 1e-8), rtol=1e-9, atol=0), step
    th, m, v = mlp.adam(np.zeros(1), np.array([2.0]), np.zeros(1), np.zeros(1), lr, 1)
    th, m, v = mlp.adam(th, np.array([-1.0]), m, v, lr, 2)
    mh, vh = 0.08 / 0.19, 0.004996 / 0.001999
    assert abs(m[0] - 0.08) < 1e-15 and abs(v[0] - 0.004996) < 1e-15
    assert abs(th[0] - (-lr * 2.0 / (2.0 + 1e-8) - lr * mh / (np.sqrt(vh) + 1e-8))) < 1e-15
