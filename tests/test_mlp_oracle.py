"""Pins of the warm-start network's CPU oracle (no GPU).

The oracle's forward, loss gradient, Adam step, bf16 rounding and twist
exponential are checked against facts outside it: central finite differences of
its own loss, an independent autograd implementation of the same network,
closed forms for degenerate weights, the Adam paper's first step, torch's
bfloat16 conversion, and the matrix exponential.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import mlp_oracle as M

torch = pytest.importorskip("torch")


def random_problem(seed=0, B=2, P=24, scale=0.5):
    rng = np.random.default_rng(seed)
    w = rng.normal(size=M.N_PARAMS) * scale
    p = M.unpack(w)
    # keep the per-point layers mostly active so the max-pool routes through them
    p["b1"][:] = np.abs(p["b1"]) + 0.1
    p["b2"][:] = np.abs(p["b2"]) + 0.1
    w = M.pack(p)
    S = [rng.normal(size=(P, 3)) for _ in range(B)]
    T = [rng.normal(size=(P, 3)) for _ in range(B)]
    Y = rng.normal(size=(B, 6))
    return w, S, T, Y


def test_layout_count():
    assert M.N_PARAMS == 64 * 3 + 64 + 128 * 64 + 128 + 128 * 256 + 128 + 6 * 128 + 6 == 42246
    w = np.arange(M.N_PARAMS, dtype=np.float64)
    assert np.array_equal(M.pack(M.unpack(w)), w)


def test_gradient_matches_central_differences():
    w, S, T, Y = random_problem(scale=0.1)          # loss O(10): FD round-off ~1e-9
    L, G = M.loss_and_grad(w, S, T, Y)
    rng = np.random.default_rng(1)
    # a sample of coordinates from every tensor
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(24, b - a), replace=False)
                          for a, b in zip(offs[:-1], offs[1:])])
    h = 1e-6
    worst = 0.0
    for k in idx:
        e = np.zeros_like(w)
        e[k] = h
        fd = (M.loss_and_grad(w + e, S, T, Y)[0] - M.loss_and_grad(w - e, S, T, Y)[0]) / (2 * h)
        worst = max(worst, abs(fd - G[k]) / (1e-3 + abs(G[k])))
    assert worst < 1e-6, worst


def test_matches_independent_autograd():
    w, S, T, Y = random_problem(seed=3, B=3, P=40)
    L, G = M.loss_and_grad(w, S, T, Y)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    parts, o = {}, 0
    for name, shp in M.SHAPES:
        n = int(np.prod(shp))
        parts[name] = wt[o:o + n].reshape(shp)
        o += n

    def feat(P):
        h1 = torch.relu(torch.as_tensor(P) @ parts["W1"].T + parts["b1"])
        h2 = torch.relu(h1 @ parts["W2"].T + parts["b2"])
        return h2.max(dim=0).values

    outs = []
    for zs, xs in zip(S, T):
        hid = torch.relu(parts["W3"] @ torch.cat([feat(zs), feat(xs)]) + parts["b3"])
        outs.append(parts["W4"] @ hid + parts["b4"])
    out = torch.stack(outs)
    loss = ((out - torch.as_tensor(Y)) ** 2).sum() / len(S)
    loss.backward()
    np.testing.assert_allclose(M.forward(w, S, T), out.detach().numpy(), rtol=1e-13, atol=1e-13)
    assert abs(L - loss.item()) <= 1e-12 * abs(L)
    np.testing.assert_allclose(G, wt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_degenerate_weights_closed_form():
    """W3 = 0: the output is W4 relu(b3) + b4 whatever the clouds, b4's gradient
    is the mean residual times two, and nothing reaches the per-point layers."""
    w, S, T, Y = random_problem(seed=5)
    p = M.unpack(w)
    p["W3"][:] = 0.0
    w = M.pack(p)
    expect = p["W4"] @ np.maximum(p["b3"], 0.0) + p["b4"]
    out = M.forward(w, S, T)
    np.testing.assert_allclose(out, np.tile(expect, (len(S), 1)), rtol=0, atol=1e-14)
    L, G = M.loss_and_grad(w, S, T, Y)
    g = M.unpack(G)
    r = expect[None, :] - Y
    np.testing.assert_allclose(g["b4"], 2 * r.sum(0) / len(S), atol=1e-14)
    np.testing.assert_allclose(g["b3"], (p["W4"].T @ (2 * r.sum(0) / len(S))) * (p["b3"] > 0), atol=1e-13)
    for name in ("W1", "b1", "W2", "b2"):
        assert not np.any(g[name]), name


def test_maxpool_routes_to_first_maximum():
    """Two identical points: only the first one carries the per-point gradient."""
    w, S, T, Y = random_problem(seed=7, B=1, P=4)
    S = [np.vstack([S[0][:1], S[0][:1], S[0][1:3]])]       # rows 0 and 1 equal
    p = M.unpack(w)
    g, arg, *_ = M.cloud_feature(S[0], p)
    assert not np.any(arg == 1)


def test_adam_first_step_is_signed_lr():
    """Kingma and Ba: after one step the bias-corrected update is
    lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    w1, m, v = M.adam_step(w0, np.zeros(4), np.zeros(4), g, step=1, lr=0.01)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, size=4000),
                        np.float32([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 65504.0])])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.bf16_round(x), ref)
    assert M.bf16_round(np.float32([1 + 2 ** -8]))[0] == 1.0           # tie to even
    assert M.bf16_round(np.float32([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


@pytest.mark.parametrize("scale", [1.0, 1e-3, 1e-9])
def test_twist_to_pose_matches_expm(scale):
    rng = np.random.default_rng(13)
    xi = rng.normal(size=6) * scale
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -xi[2], xi[1]], [xi[2], 0, -xi[0]], [-xi[1], xi[0], 0]]
    X[:3, 3] = xi[3:]
    np.testing.assert_allclose(M.twist_to_pose(xi), scipy.linalg.expm(X), atol=1e-14)
