"""The pair-grid cell size is a speed knob only: registrations with every
candidate cell fraction reach the oracle's fixed point (run on an MI355X), and
the autotuner returns one of its candidates with a timing for each."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2606_10019_amd import autotune, gcvo, synth  # noqa: E402
from tests.posemetrics import rot_err_deg, trans_err_m  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_poses.json")))


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def note(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("frac", autotune.CANDIDATES + ((0.2, 0.1), (1.0, 1.0)))
def test_every_cell_fraction_reaches_the_fixed_point(frac):
    spec = synth.make_config1(1)
    ref = GOLDEN[spec.name]
    Tref = np.array(ref["T_ref"]).reshape(4, 4)
    note(f"register config1 instance 1 with cell fraction {frac}")
    T, info = gcvo.gcvo_register(to_dev(spec.target), to_dev(spec.source), None,
                                 gcvo.params_from_spec(spec, cell_fraction=frac[0], cell_fraction_x=frac[1]))
    dr, dt = rot_err_deg(T, Tref), trans_err_m(T, Tref)
    note(f"  iters {info['iters']} (oracle {ref['prod_iters']}) err {dr:.2e} deg {dt:.2e} m")
    assert info["converged"] and dr < 1e-3 and dt < 1e-5
    assert abs(info["iters"] - ref["prod_iters"]) <= 1


def test_autotuner_returns_a_candidate():
    specs = [synth.make_config1(i) for i in (0, 2)]
    tgt = to_dev(np.concatenate([s.target for s in specs]))
    src = to_dev(np.concatenate([s.source for s in specs]))
    to = np.cumsum([0] + [len(s.target) for s in specs])
    so = np.cumsum([0] + [len(s.source) for s in specs])
    note("autotune cell fraction on two config1 pairs")
    best, timings, infos = autotune.autotune_cell_fraction(tgt, to, src, so, gcvo.params_from_spec(specs[0]), reps=1)
    note(f"  best {best}; ms per call {json.dumps({str(k): v for k, v in timings.items()})}")
    assert best in autotune.CANDIDATES and set(timings) == set(autotune.CANDIDATES)
    assert all(v > 0 for v in timings.values())
    for frac, inf in infos.items():
        assert all(i["converged"] for i in inf), frac
