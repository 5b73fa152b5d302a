"""FP64 CPU oracle of the warm-start point-set network.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never
does.  It shares no code with the GPU library.

The paper has no learned component (it warm-starts only from a constant
velocity model and names learning as future work, Sec. Conclusion); this
network is the project's own addition, and this module is its definition:

  per cloud, for each of its P input points p (already gathered, moved by the
  cloud's per-pair motion if it has one, divided by the input scale):
      h1 = relu(W1 p + b1)            3 -> 64
      h2 = relu(W2 h1 + b2)           64 -> 128
      g  = max over the P points of h2, per channel
  per pair:
      in  = [g_source, g_target]      256
      hid = relu(W3 in + b3)          256 -> 128
      out = W4 hid + b4               128 -> 6
  loss  = (1/B) sum_b ||out_b - y_b||^2

The flat parameter vector holds W1 (64x3), b1, W2 (128x64), b2, W3 (128x256),
b3, W4 (6x128), b4, each row-major, in that order.  Weights are given as
float64 arrays (bf16 values when the GPU runs them in bf16); every product and
sum here is plain float64.  relu'(0) = 0; the max-pool gradient goes to the
first point (lowest index) attaining the maximum.
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (128, 64)), ("b2", (128,)),
          ("W3", (128, 256)), ("b3", (128,)), ("W4", (6, 128)), ("b4", (6,))]
N_PARAMS = int(sum(np.prod(s) for _, s in SHAPES))


def unpack(w: np.ndarray) -> dict:
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = w[o:o + n].reshape(shp)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SHAPES])


def relu(x):
    return np.where(x > 0.0, x, 0.0)


def cloud_feature(P: np.ndarray, p: dict):
    """Per-point layers and the channel-wise max over the points of one cloud.
    Returns (g [128], argmax [128], pre1 [P, 64], h1 [P, 64], pre2 [P, 128])."""
    pre1 = P @ p["W1"].T + p["b1"]
    h1 = relu(pre1)
    pre2 = h1 @ p["W2"].T + p["b2"]
    h2 = relu(pre2)
    arg = np.argmax(pre2, axis=0)            # first index attaining the maximum
    g = h2[arg, np.arange(h2.shape[1])]
    return g, arg, pre1, h1, pre2


def gather_inputs(src_clouds, tgt_clouds, src_idx, tgt_idx, src_motion, input_scale, tgt_motion=None):
    """Input points of each pair: the chosen rows of each cloud, moved by the
    pair's 3x4 motion [R | t] for that cloud (p -> R p + t) when one is given,
    then divided by the input scale."""
    def pick(cloud, idx, motion):
        P = np.asarray(cloud, np.float64)[np.asarray(idx)]
        if motion is not None:
            M = np.asarray(motion, np.float64).reshape(3, 4)
            P = P @ M[:, :3].T + M[:, 3]
        return P / input_scale

    S, T = [], []
    for b in range(len(src_clouds)):
        S.append(pick(src_clouds[b], src_idx[b], None if src_motion is None else src_motion[b]))
        T.append(pick(tgt_clouds[b], tgt_idx[b], None if tgt_motion is None else tgt_motion[b]))
    return S, T


def forward(w, S, T):
    """Network outputs [B, 6] for per-pair input point arrays S (source) and T
    (target), each [P, 3]."""
    p = unpack(w)
    out = []
    for zs, xs in zip(S, T):
        gs = cloud_feature(zs, p)[0]
        gt = cloud_feature(xs, p)[0]
        hid = relu(p["W3"] @ np.concatenate([gs, gt]) + p["b3"])
        out.append(p["W4"] @ hid + p["b4"])
    return np.array(out)


def loss_and_grad(w, S, T, Y):
    """Loss (1/B) sum ||out - y||^2 and its gradient with respect to the flat
    parameter vector, by the chain rule written out layer by layer."""
    p = unpack(w)
    B = len(S)
    G = {name: np.zeros(shp) for name, shp in SHAPES}
    loss = 0.0
    for zs, xs, y in zip(S, T, np.asarray(Y, np.float64)):
        feats = [cloud_feature(zs, p), cloud_feature(xs, p)]
        x_in = np.concatenate([feats[0][0], feats[1][0]])
        pre3 = p["W3"] @ x_in + p["b3"]
        hid = relu(pre3)
        out = p["W4"] @ hid + p["b4"]
        r = out - y
        loss += float(r @ r) / B
        d_out = 2.0 * r / B
        G["W4"] += np.outer(d_out, hid)
        G["b4"] += d_out
        d_pre3 = (p["W4"].T @ d_out) * (pre3 > 0.0)
        G["W3"] += np.outer(d_pre3, x_in)
        G["b3"] += d_pre3
        d_in = p["W3"].T @ d_pre3
        for c, (pts, (g, arg, pre1, h1, pre2)) in enumerate(zip((zs, xs), feats)):
            d_g = d_in[128 * c:128 * (c + 1)]
            # max-pool: channel k's gradient goes to point arg[k] only
            d_pre2 = np.zeros_like(pre2)
            d_pre2[arg, np.arange(128)] = d_g * (pre2[arg, np.arange(128)] > 0.0)
            G["W2"] += d_pre2.T @ h1
            G["b2"] += d_pre2.sum(0)
            d_pre1 = (d_pre2 @ p["W2"]) * (pre1 > 0.0)
            G["W1"] += d_pre1.T @ pts
            G["b1"] += d_pre1.sum(0)
    return loss, pack(G)


def adam_step(w, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) with bias-corrected moments."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32: keep the top 16 bits of the IEEE single after adding half an ulp of
    bfloat16 plus the tie-breaking bit."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def twist_to_pose(xi: np.ndarray) -> np.ndarray:
    """exp of the twist (w, v) in closed form: Rodrigues for R and the left
    Jacobian for t, both from the series definitions (used only to check the
    GPU's pose output)."""
    w, v = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(w))
    W = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-8:
        A, Bc, C = 1.0, 0.5, 1.0 / 6.0
    else:
        A, Bc, C = np.sin(th) / th, (1 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
    R = np.eye(3) + A * W + Bc * W @ W
    V = np.eye(3) + Bc * W + C * W @ W
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ v
    return T
