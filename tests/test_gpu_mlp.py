"""BF16-MFMA surrogate kernels against the bf16-emulating fp64 reference (needs an MI355X).

Tolerances: the kernels and the reference round the same quantities to bf16;
they differ by fp32 vs fp64 arithmetic before each rounding, so an element
lying within ~1e-7 of a bf16 rounding boundary can round the other way
(probability ~1e-7 / 2^-8 per element).  One flipped element moves a 64-term
sum by at most 2^-8 of that term: outputs agree to a few 1e-3 of their scale
and gradients to 1e-2 norm-wise, far tighter than a wrong layout or a missing
term (errors of order 1)."""
import sys

import numpy as np
import pytest

import paper_1105_4840_amd as ppp
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _params(seed):
    th = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    th[mlp.H:2 * mlp.H] = rng.normal(0, 0.3, mlp.H)                     # b1
    th[2 * mlp.H + mlp.H * mlp.H:3 * mlp.H + mlp.H * mlp.H] = rng.normal(0, 0.3, mlp.H)   # b2
    th[-1] = 0.7
    return th


def _dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device="cuda")


def _fwd(th, t):
    n = len(t)
    y = torch.zeros(n, device="cuda"); dy = torch.zeros(n, device="cuda")
    P, T = _dev(th), _dev(t)          # keep the device buffers alive across the launch
    st = ppp.lib().ppp_mlp_forward(ppp._ptr(P), ppp._ptr(T), n, ppp._ptr(y), ppp._ptr(dy), ppp._stream())
    assert st == 0
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), dy.cpu().numpy().astype(np.float64)


def _grad(th, t, yv, wv, ys, ws):
    g = torch.zeros(mlp.NPARAM, device="cuda"); L = torch.zeros(1, device="cuda")
    args = [_dev(a) for a in (th, t, yv, wv, ys, ws)]
    st = ppp.lib().ppp_mlp_grad(*[ppp._ptr(a) for a in args], len(t), ppp._ptr(g), ppp._ptr(L), ppp._stream())
    assert st == 0
    return float(L.item()), g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 300, 4096])
def test_forward_matches_reference(n):
    _say(f"case mlp forward n={n}")
    th = _params(n)
    t = np.linspace(-1, 1, n) if n > 1 else np.array([0.3])
    y, dy = _fwd(th, t)
    yr, dyr, _ = mlp.forward(mlp.bf16(th.astype(np.float32)), t.astype(np.float32).astype(np.float64), True)
    sy = 1 + np.max(np.abs(yr)); sd = 1 + np.max(np.abs(dyr))
    _say(f"  max|dy| err {np.max(np.abs(y - yr)) / sy:.2e} {np.max(np.abs(dy - dyr)) / sd:.2e}")
    assert np.max(np.abs(y - yr)) <= 4e-3 * sy
    assert np.max(np.abs(dy - dyr)) <= 4e-3 * sd
    # and the plain fp64 network is within bf16 precision
    y64, dy64, _ = mlp.forward(th, t, False)
    assert np.max(np.abs(y - y64)) <= 5e-2 * sy


@pytest.mark.parametrize("n", [16, 33, 500, 4096])
def test_gradient_matches_reference(n):
    _say(f"case mlp grad n={n}")
    th = _params(7 + n)
    rng = np.random.default_rng(n)
    t = rng.uniform(-1, 1, n)
    yv = np.sin(2 * t); ys = 2 * np.cos(2 * t)
    wv = rng.uniform(0, 1, n); ws = rng.uniform(0, 1, n)
    wv[::5] = 0.0                           # value-only / slope-only points too
    L, g = _grad(th, t, yv, wv, ys, ws)
    f = lambda a: np.asarray(a, np.float32).astype(np.float64)
    Lr, gr = mlp.loss_and_grad(mlp.bf16(f(th)), f(t), f(yv), f(wv), f(ys), f(ws), True)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"  loss {L:.6g} vs {Lr:.6g}; grad rel err {rel:.2e}")
    assert abs(L - Lr) <= 1e-2 * abs(Lr)
    assert rel <= 1e-2
    # every block of the parameter vector carries its own gradient
    H = mlp.H
    for lo, hi in ((0, H), (H, 2 * H), (2 * H, 2 * H + H * H), (2 * H + H * H, 3 * H + H * H),
                   (3 * H + H * H, 4 * H + H * H), (mlp.NPARAM - 1, mlp.NPARAM)):
        assert np.linalg.norm(g[lo:hi] - gr[lo:hi]) <= 2e-2 * (np.linalg.norm(gr[lo:hi]) + 1e-3 * np.linalg.norm(gr))


def test_adam_and_training_on_gpu():
    _say("case mlp adam/training")
    th = _params(3)
    rng = np.random.default_rng(0)
    g = rng.normal(size=mlp.NPARAM)
    m0 = rng.normal(size=mlp.NPARAM) * 0.1; v0 = np.abs(rng.normal(size=mlp.NPARAM)) * 0.1
    P, G, M, V = _dev(th), _dev(g), _dev(m0), _dev(v0)
    assert ppp.lib().ppp_mlp_adam(ppp._ptr(P), ppp._ptr(G), ppp._ptr(M), ppp._ptr(V), 1e-3, 3, ppp._stream()) == 0
    torch.cuda.synchronize()
    thr, mr, vr = mlp.adam(th, g, m0, v0, 1e-3, 3)
    assert np.allclose(P.cpu().numpy(), thr, rtol=1e-5, atol=1e-6)
    assert np.allclose(M.cpu().numpy(), mr, rtol=1e-5, atol=1e-6)
    # fit F(t) = sin(2t) with slopes: the loss falls by more than an order of magnitude
    t = np.linspace(-1, 1, 200)
    T, YV, WV, YS, WS = (_dev(a) for a in (t, np.sin(2 * t), np.ones_like(t), 2 * np.cos(2 * t), 0.3 * np.ones_like(t)))
    P = _dev(_params(5)); M = torch.zeros_like(P); V = torch.zeros_like(P)
    Gd = torch.zeros_like(P); L = torch.zeros(1, device="cuda")
    losses = []
    for k in range(1, 301):
        ppp.lib().ppp_mlp_grad(ppp._ptr(P), ppp._ptr(T), ppp._ptr(YV), ppp._ptr(WV), ppp._ptr(YS), ppp._ptr(WS),
                               len(t), ppp._ptr(Gd), ppp._ptr(L), ppp._stream())
        ppp.lib().ppp_mlp_adam(ppp._ptr(P), ppp._ptr(Gd), ppp._ptr(M), ppp._ptr(V), 3e-3, k, ppp._stream())
        if k in (1, 300):
            losses.append(float(L.item()))
    _say(f"  loss {losses[0]:.4g} -> {losses[1]:.4g}")
    assert losses[1] < 0.05 * losses[0]
