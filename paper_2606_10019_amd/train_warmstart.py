"""Train the warm-start network on large-motion LiDAR pairs and evaluate it.

    python -m paper_2606_10019_amd.train_warmstart --pairs 512 --steps 4000 \
        --out paper_2606_10019_amd/weights/warmstart_lidar.npz

1. Generate the training pairs (yaw up to 15 deg, planar motion up to 3 m) on
   the host's cores.
2. Label each pair with plain G-CVO (annealed 1.0 -> 0.1 m) started at its true
   motion; the fixed point is the label.
3. Train with the library's kernels (gcvo_mlp_loss_grad + gcvo_mlp_adam); every
   sample re-poses a labelled pair by a fresh motion from the same range and
   draws fresh 1024-point subsamples (sensor-centred headings, see warmstart).
4. Evaluate on held-out pairs: prediction error, and plain registration from
   identity vs the warm-started one, against the plain solver's fixed point from
   the true motion.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import gcvo, synth, warmstart


def _make(args):
    i, split = args
    return synth.make_config5(i, split)


def generate(n: int, split: str, workers: int):
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_make, [(i, split) for i in range(n)], chunksize=4))


def rot_deg(Ta, Tb):
    dR = Ta[:3, :3].T @ Tb[:3, :3]
    return float(np.degrees(np.arctan2(np.linalg.norm([dR[2, 1] - dR[1, 2], dR[0, 2] - dR[2, 0],
                                                       dR[1, 0] - dR[0, 1]]) / 2, (np.trace(dR) - 1) / 2)))


def label(specs, chunk: int = 64):
    """Plain G-CVO from the true motion, in batches; returns (T [n,4,4], converged)."""
    Ts, conv = [], []
    for a in range(0, len(specs), chunk):
        part = specs[a:a + chunk]
        ps = warmstart.PairSet.from_specs(part)
        T, infos = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off,
                                            np.array([s.T_true for s in part]),
                                            [gcvo.params_from_spec(s) for s in part])
        Ts.extend(T)
        conv.extend(i["converged"] for i in infos)
    return np.array(Ts), np.array(conv)


def evaluate(net, specs, refs, log, refine_length_scale=None):
    """Plain from identity vs warm-started, both batched, judged against refs
    (plain solver from the true motion) at 1e-3 deg / 1e-5 m."""
    import torch
    ps = warmstart.PairSet.from_specs(specs)
    params = [gcvo.params_from_spec(s) for s in specs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tp, ip = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off, None, params)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    Tw, iw, rec = warmstart.register_warm(net, ps, params, refine_length_scale)
    Tw = Tw.cpu().numpy()
    t_warm = time.perf_counter() - t0
    rec["T0"] = rec["T0"].cpu().numpy()

    def ok(T, info, R):
        return info["converged"] and rot_deg(T, R) <= 1e-3 and np.linalg.norm(T[:3, 3] - R[:3, 3]) <= 1e-5

    n_plain = sum(ok(Tp[k], ip[k], refs[k]) for k in range(len(specs)))
    n_warm = sum(ok(Tw[k], iw[k], refs[k]) for k in range(len(specs)))
    pe = [(rot_deg(rec["T0"][k], refs[k]), float(np.linalg.norm(rec["T0"][k][:3, 3] - refs[k][:3, 3])))
          for k in range(len(specs))]
    res = dict(pairs=len(specs), plain_in_gate=int(n_plain), warm_in_gate=int(n_warm), plain_s=t_plain, warm_s=t_warm,
               plain_iters=float(np.mean([i["iters"] for i in ip])), warm_iters=float(np.mean([i["iters"] for i in iw])),
               fallbacks=len(rec["fallback"]), pred_rot_err_deg_median=float(np.median([p[0] for p in pe])),
               pred_trans_err_m_median=float(np.median([p[1] for p in pe])),
               pred_rot_err_deg_p90=float(np.percentile([p[0] for p in pe], 90)),
               pred_trans_err_m_p90=float(np.percentile([p[1] for p in pe], 90)),
               refine_length_scale=refine_length_scale)
    log(json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=512)
    ap.add_argument("--eval-pairs", type=int, default=64)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=warmstart.WEIGHTS)
    args = ap.parse_args()

    def log(msg):
        print(f"[train] {msg}", flush=True)

    t0 = time.time()
    train_specs = generate(args.pairs, "train", args.workers)
    eval_specs = generate(args.eval_pairs, "eval", args.workers)
    log(f"generated {len(train_specs)} + {len(eval_specs)} pairs in {time.time() - t0:.1f} s")
    import torch
    dev = torch.device("cuda:0")
    t0 = time.time()
    labels, conv = label(train_specs)
    refs, rconv = label(eval_specs)
    truth_err = [rot_deg(labels[k], s.T_true) for k, s in enumerate(train_specs)]
    log(f"labelled in {time.time() - t0:.1f} s; converged {int(conv.sum())}/{len(conv)}; "
        f"median label-vs-truth {np.median(truth_err):.3f} deg")
    keep = np.nonzero(conv)[0]
    ps = warmstart.PairSet.from_specs([train_specs[k] for k in keep], dev)
    net = warmstart.Network(warmstart.Network.init_weights(args.seed), dev)
    t0 = time.time()
    losses = warmstart.train(net, ps, labels[keep], args.steps, args.batch, args.lr, args.lr_final, seed=args.seed,
                             log=log, log_every=max(200, args.steps // 20))
    t_train = time.time() - t0
    log(f"trained {args.steps} steps x {args.batch} in {t_train:.1f} s")
    ev_keep = [k for k in range(len(eval_specs)) if rconv[k]]
    results = [evaluate(net, [eval_specs[k] for k in ev_keep], refs[ev_keep], log, ell) for ell in (None, 0.5)]
    meta = dict(pairs=int(len(keep)), steps=args.steps, batch=args.batch, lr=args.lr, lr_final=args.lr_final,
                seed=args.seed, crop_m=warmstart.CROP_M,
                samples=args.steps * args.batch, input_scale=warmstart.INPUT_SCALE, n_points=warmstart.N_POINTS,
                final_loss=float(np.mean(losses[-100:])), first_loss=float(np.mean(losses[:100])),
                train_seconds=t_train, eval=results)
    net.save(args.out, meta)
    log(f"saved {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
