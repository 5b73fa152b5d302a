"""The stored oracle poses still describe the inputs the generators produce.

A generator drift (numpy, scipy or code change) would make every GPU-vs-oracle
comparison meaningless, so the digests of the float32 clouds are checked, and
one stored pose is recomputed by the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_10019_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_poses.json")


def load():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_golden_digests_match_generators():
    data = load()
    names = [k for k in data if not k.startswith("_")]
    assert len(names) >= 12
    for name in names:
        e = data[name]
        if e["config"] in (2, 3, 5) and e["instance"] > 0:
            continue  # covered by instance 0; each ray-cast scene takes seconds
        if e["config"] == 5:
            spec = synth.make_config5(e["instance"], e.get("split", "train"))
        else:
            spec = synth.make_pair(e["config"], e["instance"])
        assert spec.name == name.split("/")[0]     # "<pair>/<variant>" entries share the pair's inputs
        assert spec.digest() == e["digest"], f"generator drift for {name}"


def test_golden_pose_reproduces():
    e = load()["c1_planes_cap_0"]
    spec = synth.make_pair(1, 0)
    r = O.register_spec(spec, tol=1e-12, max_iters=500)
    np.testing.assert_allclose(r.T.reshape(-1), np.array(e["T_ref"]), atol=1e-12)
    assert r.iters == e["ref_iters"]
