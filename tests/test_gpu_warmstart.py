"""The trained warm start against plain registration from identity (run on an
MI355X).

Held-out large-motion LiDAR pairs (yaw up to 15 deg, planar motion up to 3 m,
about 30k points per cloud).  The reference pose of each pair is the FP64
oracle's fixed point reached from the true motion with the pair's annealing
schedule (``tests/golden/oracle_poses.json``, written by the oracle only).  A
registration counts when it converged within 1e-3 deg / 1e-5 m of that
reference.  The committed network must turn substantially more of these pairs
into correct registrations than the plain solver from identity, at no more
solver iterations on average (within one): at least a quarter of the pairs more within the gate,
and at least 1.5 times as many as the plain solver.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2606_10019_amd import gcvo, synth, warmstart  # noqa: E402
from tests.posemetrics import rot_err_deg, trans_err_m  # noqa: E402

pytestmark = pytest.mark.gpu
N_PAIRS = 24
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_poses.json")))


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def oracle_refs(specs):
    refs = []
    for s in specs:
        g = GOLDEN.get(s.name)
        assert g is not None, f"no oracle reference for {s.name} (run tests/golden/make_golden.py --c5-eval)"
        assert g["digest"] == s.digest(), f"{s.name}: input drifted from the stored reference"
        refs.append((np.array(g["T_ref"]).reshape(4, 4), bool(g["ref_converged"])))
    return refs


def test_warm_start_gain_over_plain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    specs = [synth.make_config5(i, "eval") for i in range(N_PAIRS)]
    refs = oracle_refs(specs)
    keep = [k for k in range(N_PAIRS) if refs[k][1]]
    note(f"warm start: {N_PAIRS} held-out pairs ({np.mean([len(s.source) for s in specs]):.0f} points per "
         f"cloud), {len(keep)} with a converged oracle reference")
    ps = warmstart.PairSet.from_specs(specs, dev)
    params = [gcvo.params_from_spec(s) for s in specs]
    Tp, ip = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off, None, params)
    net = warmstart.Network.load(device=dev)
    Tw, iw, rec = warmstart.register_warm(net, ps, params)
    assert Tw.is_cuda and rec["T0"].is_cuda            # poses never leave the device on the way
    Tw, T0 = Tw.cpu().numpy(), rec["T0"].cpu().numpy()

    def ok(T, info, R):
        return info["converged"] and rot_err_deg(T, R) <= 1e-3 and trans_err_m(T, R) <= 1e-5

    plain = sum(ok(Tp[k], ip[k], refs[k][0]) for k in keep)
    warm = sum(ok(Tw[k], iw[k], refs[k][0]) for k in keep)
    pred_rot = np.median([rot_err_deg(T0[k], refs[k][0]) for k in keep])
    pred_tr = np.median([trans_err_m(T0[k], refs[k][0]) for k in keep])
    it_p = np.mean([ip[k]["iters"] for k in keep])
    it_w = np.mean([iw[k]["iters"] for k in keep])
    note(f"  plain {plain}/{len(keep)} in gate ({it_p:.1f} iters); warm {warm}/{len(keep)} ({it_w:.1f} iters), "
         f"{len(rec['fallback'])} fallbacks; prediction median error {pred_rot:.2f} deg {pred_tr:.2f} m")
    assert warm >= plain + len(keep) // 4
    assert warm >= 1.5 * plain
    assert it_w <= it_p + 1
