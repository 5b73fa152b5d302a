"""The trained warm start against plain registration from identity (run on an
MI355X).

Held-out large-motion LiDAR pairs (yaw up to 15 deg, planar motion up to 3 m):
the reference pose of each pair is plain G-CVO's fixed point started at the
true motion (the solver judges the error).  A registration counts when it is
within 1e-3 deg / 1e-5 m of that reference.  The committed network must turn
substantially more of these pairs into correct registrations than the plain
solver from identity, at no more solver iterations.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2606_10019_amd import gcvo, synth, warmstart  # noqa: E402
from tests.posemetrics import rot_err_deg, trans_err_m  # noqa: E402

pytestmark = pytest.mark.gpu
N_PAIRS = 24


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def test_warm_start_gain_over_plain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    specs = [synth.make_config5(i, "eval") for i in range(N_PAIRS)]
    ps = warmstart.PairSet.from_specs(specs, dev)
    params = [gcvo.params_from_spec(s) for s in specs]
    refs, rinfo = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off,
                                           np.array([s.T_true for s in specs]), params)
    keep = [k for k in range(N_PAIRS) if rinfo[k]["converged"]]
    note(f"warm start: {N_PAIRS} held-out pairs, {len(keep)} with a converged reference")
    Tp, ip = gcvo.gcvo_register_batch(ps.targets, ps.tgt_off, ps.sources, ps.src_off, None, params)
    net = warmstart.Network.load(device=dev)
    Tw, iw, rec = warmstart.register_warm(net, ps, params)

    def ok(T, info, R):
        return info["converged"] and rot_deg_ok(T, R)

    def rot_deg_ok(T, R):
        return rot_err_deg(T, R) <= 1e-3 and trans_err_m(T, R) <= 1e-5

    plain = sum(ok(Tp[k], ip[k], refs[k]) for k in keep)
    warm = sum(ok(Tw[k], iw[k], refs[k]) for k in keep)
    pred_rot = np.median([rot_err_deg(rec["T0"][k], refs[k]) for k in keep])
    pred_tr = np.median([trans_err_m(rec["T0"][k], refs[k]) for k in keep])
    it_p = np.mean([ip[k]["iters"] for k in keep])
    it_w = np.mean([iw[k]["iters"] for k in keep])
    note(f"  plain {plain}/{len(keep)} in gate ({it_p:.1f} iters); warm {warm}/{len(keep)} ({it_w:.1f} iters), "
         f"{len(rec['fallback'])} fallbacks; prediction median error {pred_rot:.2f} deg {pred_tr:.2f} m")
    assert warm >= plain + len(keep) // 4
    assert warm >= 0.7 * len(keep)
    assert it_w <= it_p
