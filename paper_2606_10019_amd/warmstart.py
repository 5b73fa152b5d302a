"""Learned warm start for LiDAR registration: data, training loop and the
warm-started registration with its fallback.

The network and its training arithmetic run in the library's HIP kernels
(``gcvo_mlp_*``, see ``include/gcvo_mlp.h``); this module only prepares host
data (which rows to feed, which motion re-poses a training pair, the label
twists) and sequences the calls.

Labels come from the registration method itself: each training pair is solved
by plain G-CVO started at its true motion, and its fixed point is the label.  A
training sample turns the target cloud by R1 and the source cloud by R2, both
rotations about the vertical axis through the cloud's own sensor (so each
cloud still sits in a sensor-centred frame, as at inference).  The objective
and the per-point covariances are equivariant under these motions, so the
fixed point becomes exactly R2 T R1^{-1}; R1 is uniform in heading and R2 is
chosen so that the new relative yaw is uniform in the workload's range.

The network sees a 1024-point subsample of the points within CROP_M metres
(horizontally) of each sensor.

Warm-started registration: the network predicts T0 from those subsamples,
plain G-CVO refines from T0 with the pair's annealing schedule (optionally
starting at a smaller length scale), and the result is kept unless the refine
did not converge or its objective is below the objective at T = I, both
evaluated at the schedule's first length scale (two evaluations); then the
plain solver from identity is run and its result returned.  The comparison is
made at the first length scale because at the final one the objective of two
scans from a spinning sensor peaks at T = I, where the scan rings coincide,
whatever the true motion.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

from . import gcvo

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "warmstart_lidar.npz")
N_POINTS = 1024
INPUT_SCALE = 40.0
MAX_YAW_DEG = 15.0
MAX_TRANS_M = 3.0
CROP_M = 80.0

SHAPES = [(64, 3), (64,), (128, 64), (128,), (128, 256), (128,), (6, 128), (6,)]


# ------------------------------------------------------------------ SE(3) host helpers

def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_log(T: np.ndarray) -> np.ndarray:
    """Twist (w, v) with exp(xi^) = T, for rotation angles below pi."""
    R, t = T[:3, :3], T[:3, 3]
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    if th < 1e-6:
        w = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]]) / 2.0
        W = hat(w)
        Vinv = np.eye(3) - 0.5 * W + W @ W / 12.0
    else:
        w = th / (2.0 * np.sin(th)) * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
        W = hat(w)
        Vinv = np.eye(3) - 0.5 * W + (1.0 / th ** 2) * (1.0 - (th * np.sin(th)) / (2.0 * (1.0 - np.cos(th)))) * W @ W
    return np.concatenate([w, Vinv @ t])


def planar_motion(rng: np.random.Generator, max_yaw_deg=MAX_YAW_DEG, max_trans_m=MAX_TRANS_M) -> np.ndarray:
    """Ego motion of the workload: yaw U[-15, 15] deg, planar translation of
    U[0, 3] m in a uniform direction."""
    yaw = np.deg2rad(rng.uniform(-max_yaw_deg, max_yaw_deg))
    phi = rng.uniform(0.0, 2.0 * np.pi)
    d = rng.uniform(0.0, max_trans_m)
    T = np.eye(4)
    T[:2, :2] = [[np.cos(yaw), -np.sin(yaw)], [np.sin(yaw), np.cos(yaw)]]
    T[:3, 3] = [d * np.cos(phi), d * np.sin(phi), 0.0]
    return T


def normalised_twist(T: np.ndarray) -> np.ndarray:
    xi = se3_log(T)
    return np.concatenate([xi[:3] / gcvo.GCVO_MLP_ROT_SCALE, xi[3:] / gcvo.GCVO_MLP_TRANS_SCALE])


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 (ties to even) of float32 values, as raw uint16 bits."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


# ------------------------------------------------------------------ network state

class Network:
    """FP32 master weights, the bfloat16 copy the kernels read, Adam moments."""

    def __init__(self, master: np.ndarray, device="cuda"):
        import torch
        master = np.ascontiguousarray(master, np.float32)
        assert master.shape == (gcvo.GCVO_MLP_N_PARAMS,)
        self.device = torch.device(device)
        self.w = torch.from_numpy(master.copy()).to(self.device)
        self.wb = torch.from_numpy(bf16_bits(master).view(np.int16)).to(self.device)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.step = 0

    @staticmethod
    def init_weights(seed: int = 0) -> np.ndarray:
        """He-uniform weights, zero biases."""
        rng = np.random.default_rng(seed)
        parts = []
        for shp in SHAPES:
            if len(shp) == 2:
                lim = np.sqrt(6.0 / shp[1])
                parts.append(rng.uniform(-lim, lim, size=shp).reshape(-1))
            else:
                parts.append(np.zeros(shp))
        return np.concatenate(parts).astype(np.float32)

    @classmethod
    def load(cls, path: str = WEIGHTS, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            net = cls(z["master"], device)
            net.meta = json.loads(str(z["meta"]))
        return net

    def save(self, path: str, meta: dict) -> None:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, master=self.w.cpu().numpy(), meta=json.dumps(meta))


# ------------------------------------------------------------------ training data

@dataclass
class PairSet:
    """Clouds of several pairs concatenated on the device, with host offsets
    and, per cloud, the rows the network may see (within the crop radius)."""
    targets: object
    sources: object
    tgt_off: np.ndarray
    src_off: np.ndarray
    tgt_rows: list
    src_rows: list

    @classmethod
    def from_specs(cls, specs, device="cuda", crop_m: float = CROP_M):
        import torch
        dev = torch.device(device)
        tgt = torch.from_numpy(np.concatenate([s.target for s in specs])).to(dev)
        src = torch.from_numpy(np.concatenate([s.source for s in specs])).to(dev)
        to = np.cumsum([0] + [len(s.target) for s in specs]).astype(np.int64)
        so = np.cumsum([0] + [len(s.source) for s in specs]).astype(np.int64)

        def rows(P):
            r = np.nonzero(np.hypot(P[:, 0], P[:, 1]) <= crop_m)[0] if crop_m else np.arange(len(P))
            return r if len(r) else np.arange(len(P))

        return cls(tgt, src, to, so, [rows(s.target) for s in specs], [rows(s.source) for s in specs])

    @property
    def n(self) -> int:
        return len(self.tgt_off) - 1


def subsample_indices(rng: np.random.Generator, eligible, n_points: int = N_POINTS) -> np.ndarray:
    """Rows fed to the network: n_points distinct eligible rows per cloud when
    it has that many, else eligible rows drawn with replacement."""
    out = np.empty((len(eligible), n_points), np.int32)
    for k, rows in enumerate(eligible):
        out[k] = rows[rng.choice(len(rows), size=n_points, replace=len(rows) < n_points)]
    return out


def _motion_rows(Ts):
    import torch
    return None if Ts is None else torch.from_numpy(np.ascontiguousarray(
        np.asarray(Ts)[:, :3, :].reshape(-1, 12), np.float32))


def batch_inputs(ps: PairSet, pair_ids, rng: np.random.Generator, tgt_motions=None, src_motions=None,
                 n_points: int = N_POINTS):
    """An MlpBatch for the chosen pairs of the set (repeats allowed): each
    sample reads its pair's row ranges and a fresh subsample of eligible rows."""
    import torch
    dev = ps.targets.device
    ids = np.asarray(pair_ids)
    ts, tc = ps.tgt_off[ids], (ps.tgt_off[1:] - ps.tgt_off[:-1])[ids]
    ss, sc = ps.src_off[ids], (ps.src_off[1:] - ps.src_off[:-1])[ids]
    tidx = torch.from_numpy(subsample_indices(rng, [ps.tgt_rows[b] for b in ids], n_points)).to(dev)
    sidx = torch.from_numpy(subsample_indices(rng, [ps.src_rows[b] for b in ids], n_points)).to(dev)
    tm, sm = _motion_rows(tgt_motions), _motion_rows(src_motions)
    return gcvo.MlpBatch(ps.targets, ts, tc, ps.sources, ss, sc, tidx, sidx,
                         tm.to(dev) if tm is not None else None, sm.to(dev) if sm is not None else None, INPUT_SCALE)


def yaw_rotation(a: float) -> np.ndarray:
    T = np.eye(4)
    T[:2, :2] = [[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]]
    return T


def train(net: Network, ps: PairSet, labels: np.ndarray, steps: int, batch: int = 64, lr: float = 1e-3,
          lr_final: float = 1e-5, seed: int = 0, log_every: int = 200, log=None):
    """Adam on the twist regression loss.  Every step draws `batch` labelled
    pairs, per sample a heading R1 for the target (uniform) and R2 for the
    source such that the new label R2 T R1^{-1} has a yaw uniform in the
    workload's range, and fresh 1024-point subsamples.  Returns the per-step
    losses (host floats, read back every log_every steps)."""
    import torch
    rng = np.random.default_rng(seed)
    yaws = np.arctan2(labels[:, 1, 0], labels[:, 0, 0])
    max_yaw = np.deg2rad(MAX_YAW_DEG)
    losses = []
    pending = []
    for k in range(steps):
        ids = rng.integers(0, ps.n, size=batch)
        r1 = rng.uniform(-np.pi, np.pi, size=batch)
        r2 = r1 + rng.uniform(-max_yaw, max_yaw, size=batch) - yaws[ids]
        R1 = [yaw_rotation(a) for a in r1]
        R2 = [yaw_rotation(a) for a in r2]
        new = [B2 @ labels[b] @ B1.T for B1, B2, b in zip(R1, R2, ids)]
        y = torch.from_numpy(np.array([normalised_twist(Tn) for Tn in new], np.float32)).to(net.device)
        bi = batch_inputs(ps, ids, rng, R1, R2)
        loss, grad = gcvo.gcvo_mlp_loss_grad(bi, net.wb, y)
        net.step += 1
        cur = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
        gcvo.gcvo_mlp_adam(net.w, net.wb, net.m, net.v, grad, net.step, cur)
        pending.append(loss)
        if (k + 1) % log_every == 0 or k + 1 == steps:
            vals = torch.cat(pending).cpu().numpy().tolist()
            losses.extend(vals)
            pending = []
            if log:
                log(f"step {k + 1}/{steps} loss {np.mean(vals):.4f} lr {cur:.2e}")
    return losses


# ------------------------------------------------------------------ warm-started registration

def predict(net: Network, ps: PairSet, seed: int = 0):
    """Predicted registration poses of every pair of the set (float64 CUDA
    tensor [B, 4, 4]: they stay on the device as the refine's start poses)."""
    rng = np.random.default_rng(seed)
    bi = batch_inputs(ps, np.arange(ps.n), rng)
    _, T = gcvo.gcvo_mlp_forward(bi, net.wb, poses=True)
    return T


def _params_copy(p, **kw):
    q = gcvo.gcvo_params()
    for name, _ in gcvo.gcvo_params._fields_:
        setattr(q, name, getattr(p, name))
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def objective_at(ps: PairSet, shapes, poses, length_scales, params):
    """f of every pair at the given poses (None: identity; a float64 CUDA
    tensor [B, 4, 4] otherwise) with each pair's length scale, from one batched
    evaluation over the pairs' shapes (a (target, source) pair of
    gcvo_point_shapes_batch outputs).  Device float64 [B]."""
    p0 = params[0]
    return gcvo.gcvo_eval_fgh_batch(ps.targets, shapes[0], ps.tgt_off, ps.sources, shapes[1], ps.src_off, poses,
                                    length_scales, p0.cutoff_scale, p0.sigma2, p0.precision).f


def _subset(ps: PairSet, ids):
    """The clouds of the chosen pairs, concatenated anew on the device."""
    import torch
    t = torch.cat([ps.targets[ps.tgt_off[k]:ps.tgt_off[k + 1]] for k in ids])
    s = torch.cat([ps.sources[ps.src_off[k]:ps.src_off[k + 1]] for k in ids])
    to = np.cumsum([0] + [int(ps.tgt_off[k + 1] - ps.tgt_off[k]) for k in ids]).astype(np.int64)
    so = np.cumsum([0] + [int(ps.src_off[k + 1] - ps.src_off[k]) for k in ids]).astype(np.int64)
    return t, to, s, so


def register_warm(net: Network, ps: PairSet, params, refine_length_scale: float | None = None, seed: int = 0):
    """Warm-started batch registration with the objective fallback.  params:
    one gcvo_params per pair (the plain schedule); refine_length_scale, when
    given, starts the refine's schedule there instead.  The predicted poses,
    the refined poses and the objectives stay on the device; the host reads
    back only the run summaries and two objectives per pair to pick the
    fallbacks.  Returns (T float64 CUDA [B, 4, 4], infos, record) where record
    holds the predictions, which pairs fell back, and the two objectives."""
    import torch
    T0 = predict(net, ps, seed)
    rp = [p if refine_length_scale is None else
          _params_copy(p, length_scale=max(min(refine_length_scale, p.length_scale), p.length_scale_min))
          for p in params]
    T, info_dev = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off, T0, rp, device=True)
    p0 = params[0]
    shapes = (gcvo.gcvo_point_shapes_batch(ps.targets, ps.tgt_off, p0.knn, p0.eig_ratio_min),
              gcvo.gcvo_point_shapes_batch(ps.sources, ps.src_off, p0.knn, p0.eig_ratio_min))
    ell0 = np.array([p.length_scale for p in params])
    f_ref = objective_at(ps, shapes, T, ell0, params)
    f_id = objective_at(ps, shapes, None, ell0, params)
    infos = gcvo.infos_from_device(info_dev)
    fr, fi = f_ref.cpu().numpy(), f_id.cpu().numpy()
    fall = [k for k in range(ps.n) if not infos[k]["converged"] or fr[k] < fi[k]]
    if fall:
        t, to, s, so = _subset(ps, fall)
        Tf, info_f = gcvo.gcvo_register_batch(t, to, s, so, None, [params[k] for k in fall], device=True)
        idx = torch.as_tensor(fall, device=T.device)
        T[idx] = Tf
        for r, k in enumerate(gcvo.infos_from_device(info_f)):
            infos[fall[r]] = k
    return T, infos, dict(T0=T0, fallback=fall, f_refined=fr.tolist(), f_identity=fi.tolist())
