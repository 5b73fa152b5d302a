"""Write the oracle's reference poses for the seeded synthetic pairs.

Run from the repository root:  python tests/golden/make_golden.py [--configs 1 2]

Every stored value comes from the FP64 CPU oracle (``oracle/``) applied to the
inputs of ``paper_2606_10019_amd.synth``; nothing here touches the GPU library.
The reference run uses the pair's own settings except that the final stage is
driven to ||xi||_1 < 1e-12 (cap 500 iterations), which defines the oracle's
fixed point that GPU poses are judged against.  Each entry stores the digest of
the float32 input clouds so a generator drift is detected instead of silently
comparing different problems.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2606_10019_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_poses.json")
# Object pairs: the oracle-checked sample of the 256-pair batch is every pair
# whose natural size is at most 4000 points.
C4_SAMPLE_MAX_N = 4000
INSTANCES = {1: range(8), 2: range(4), 3: range(2),
             4: [i for i, n in enumerate(synth.config4_sizes()) if n <= C4_SAMPLE_MAX_N]}


def rot_err_deg(Ta, Tb):
    dR = Ta[:3, :3].T @ Tb[:3, :3]
    return float(np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, nargs="*", default=[1, 2])
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    data["_about"] = ("FP64 oracle fixed points (final stage to ||xi||_1 < 1e-12) for the seeded "
                      "synthetic pairs; written by tests/golden/make_golden.py from oracle/ only.")
    for c in args.configs:
        for i in INSTANCES[c]:
            spec = synth.make_pair(c, i)
            t0 = time.time()
            prod = O.register_spec(spec)
            ref = O.register_spec(spec, tol=1e-12, max_iters=500)
            dt = time.time() - t0
            data[spec.name] = dict(
                config=c, instance=i, digest=spec.digest(), n_target=len(spec.target),
                n_source=len(spec.source), params=spec.params(),
                T_ref=ref.T.reshape(-1).tolist(), ref_iters=ref.iters, ref_converged=ref.converged,
                ref_stage_iters=ref.stage_iters, f_ref=ref.f, pairs_last=ref.pairs_last,
                prod_iters=prod.iters, prod_stage_iters=prod.stage_iters, prod_converged=prod.converged,
                T_prod=prod.T.reshape(-1).tolist(),
                truth_rot_deg=rot_err_deg(ref.T, spec.T_true),
                truth_trans_m=float(np.linalg.norm(ref.T[:3, 3] - spec.T_true[:3, 3])))
            print(f"{spec.name}: n={len(spec.target)}/{len(spec.source)} iters={prod.iters} "
                  f"stages={prod.stage_iters} ref_iters={ref.iters} "
                  f"truth {data[spec.name]['truth_rot_deg']:.4f} deg "
                  f"{data[spec.name]['truth_trans_m']:.4f} m  ({dt:.1f} s)", flush=True)
            with open(OUT, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
