"""GPU labelled objective (c_ij = <l^X_i, l^Z_j>, eq. rkhs_loss) and the
isotropic pair kernel (Remark 3, eig_ratio_min = 1) vs the FP64 CPU oracle,
through the C ABI (run on an MI355X).

Labels come from ``synth.pair_labels``: smooth colour channels in (0.1, 0.9) or
one-hot classes of a partition of the surface.  Tolerances are those of the
unlabelled parity tests: single evaluations within 64 eps32 / rho of each
quantity's natural scale (FP32) or 1e-11 (FP64); poses within 1e-3 deg and
1e-5 m of the oracle's fixed point.  Colour weights lie in (0.01, 2.5), so the
relative error bound of the FP32 sums is unchanged up to the label dot
product's own rounding (a few eps32).
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2606_10019_amd import gcvo, synth  # noqa: E402
from tests.posemetrics import rot_err_deg, trans_err_m  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_poses.json")))
EPS32 = float(np.finfo(np.float32).eps)
ROT_GATE_DEG, TRANS_GATE_M = 1e-3, 1e-5
FP32, FP64 = gcvo.GCVO_PRECISION_FP32, gcvo.GCVO_PRECISION_FP64


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def note(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def c1():
    spec = synth.make_config1(0)
    SX = O.point_shapes(spec.target, 10, spec.eig_ratio_min).astype(np.float32)
    SZ = O.point_shapes(spec.source, 10, spec.eig_ratio_min).astype(np.float32)
    return spec, SX, SZ


def _f64(a):
    return np.asarray(a, np.float64)


@pytest.mark.parametrize("precision", [FP32, FP64])
@pytest.mark.parametrize("kind,dim", [("colour", 3), ("class", 4), ("colour", 1)])
def test_labeled_eval_matches_oracle(c1, kind, dim, precision):
    spec, SX, SZ = c1
    LX, LZ = synth.pair_labels(spec, dim, kind)
    T = np.array(GOLDEN[spec.name]["T_ref"]).reshape(4, 4)
    note(f"eval_fgh_labeled config1 {kind} dim {dim} precision {precision}")
    g = gcvo.gcvo_eval_fgh_labeled(to_dev(spec.target), to_dev(SX.T), to_dev(LX), to_dev(spec.source), to_dev(SZ.T),
                                   to_dev(LZ), T, 0.3, 0.9, 1.0, precision)
    o = O.evaluate(_f64(spec.target), _f64(SX), _f64(spec.source), _f64(SZ), T, 0.3, 0.9, LX=_f64(LX), LZ=_f64(LZ))
    tol = 64 * EPS32 / spec.eig_ratio_min if precision == FP32 else 1e-11
    note(f"  f {g.f:.9g} vs {o.f:.9g}; pairs {g.npairs} vs {o.npairs}; "
         f"|dg|/(f/ell) {np.max(np.abs(g.g - o.g)) / (o.f / 0.3):.2e}; "
         f"|dH|/max|H| {np.max(np.abs(g.H - o.H_gn)) / np.max(np.abs(o.H_gn)):.2e}; tol {tol:.1e}")
    if precision == FP64:
        assert g.npairs == o.npairs
    else:
        assert abs(g.npairs - o.npairs) <= 2
    assert abs(g.f - o.f) <= tol * o.f
    assert np.max(np.abs(g.g - o.g)) <= tol * o.f / 0.3
    assert np.max(np.abs(g.H - o.H_gn)) <= tol * np.max(np.abs(o.H_gn))


def test_unit_and_zero_labels(c1):
    """Unit labels reproduce the unlabelled sums (the weight multiplies exactly
    by one); zero labels give f = 0, g = 0, H = 0 over the same pairs."""
    spec, SX, SZ = c1
    T = np.array(GOLDEN[spec.name]["T_ref"]).reshape(4, 4)
    tx, sx, ts, ss = to_dev(spec.target), to_dev(spec.source), to_dev(SX.T), to_dev(SZ.T)
    note("eval_fgh_labeled unit / zero labels")
    plain = gcvo.gcvo_eval_fgh(tx, ts, sx, ss, T, 0.3, 0.9)
    one = gcvo.gcvo_eval_fgh_labeled(tx, ts, to_dev(np.ones((len(spec.target), 1))), sx, ss,
                                     to_dev(np.ones((len(spec.source), 1))), T, 0.3, 0.9)
    assert one.npairs == plain.npairs
    assert abs(one.f - plain.f) <= 4 * EPS32 * plain.f
    assert np.max(np.abs(one.g - plain.g)) <= 4 * EPS32 * plain.f / 0.3
    assert np.max(np.abs(one.H - plain.H)) <= 4 * EPS32 * np.max(np.abs(plain.H))
    zero = gcvo.gcvo_eval_fgh_labeled(tx, ts, to_dev(np.zeros((len(spec.target), 2))), sx, ss,
                                      to_dev(np.ones((len(spec.source), 2))), T, 0.3, 0.9)
    assert zero.npairs == plain.npairs and zero.f == 0.0
    assert np.all(zero.g == 0.0) and np.all(zero.H == 0.0)


@pytest.mark.parametrize("kind,dim", [("colour", 3), ("class", 4)])
def test_labeled_register_batch_matches_oracle(kind, dim):
    specs = [synth.make_config1(i) for i in (0, 1)]
    labels = [synth.pair_labels(s, dim, kind) for s in specs]
    note(f"register_batch_labeled 2 config1 pairs, {kind} dim {dim}")
    tgt = np.concatenate([s.target for s in specs])
    src = np.concatenate([s.source for s in specs])
    to = np.cumsum([0] + [len(s.target) for s in specs])
    so = np.cumsum([0] + [len(s.source) for s in specs])
    LX = np.concatenate([lab[0] for lab in labels])
    LZ = np.concatenate([lab[1] for lab in labels])
    T, infos = gcvo.gcvo_register_batch_labeled(to_dev(tgt), to_dev(LX), to, to_dev(src), to_dev(LZ), so, None,
                                                gcvo.params_from_spec(specs[0]))
    for k, s in enumerate(specs):
        r = O.register_spec(s, LX=_f64(labels[k][0]), LZ=_f64(labels[k][1]))
        dr, dt = rot_err_deg(T[k], r.T), trans_err_m(T[k], r.T)
        note(f"  pair {k}: iters {infos[k]['iters']} (oracle {r.iters}) err {dr:.2e} deg {dt:.2e} m")
        assert r.converged and infos[k]["converged"]
        assert dr < ROT_GATE_DEG and dt < TRANS_GATE_M


ISO = dict(eig_ratio_min=1.0, max_iters=300, max_iters_per_stage=300)


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_isotropic_register_matches_oracle(precision):
    spec = synth.make_config1(1)
    note(f"register isotropic (rho = 1) config1 instance 1, precision {precision}")
    T, info = gcvo.gcvo_register(to_dev(spec.target), to_dev(spec.source), None,
                                 gcvo.params_from_spec(spec, precision=precision, **ISO))
    r = O.register_spec(spec, **ISO)
    dr, dt = rot_err_deg(T, r.T), trans_err_m(T, r.T)
    note(f"  iters {info['iters']} (oracle {r.iters}) pairs {info['pairs_last']} (oracle {r.pairs_last}) "
         f"err {dr:.2e} deg {dt:.2e} m")
    assert r.converged and info["converged"]
    assert dr < ROT_GATE_DEG and dt < TRANS_GATE_M
    if precision == FP64:
        assert abs(info["iters"] - r.iters) <= 1


def test_isotropic_labeled_and_mixed_batch():
    """A batch holding an isotropic labelled pair and an anisotropic labelled
    pair runs the general kernel (identity shapes for the isotropic one); both
    reach their oracle fixed points, and the isotropic pair alone (isotropic
    kernel) agrees with it."""
    specs = [synth.make_config1(2), synth.make_config1(3)]
    labels = [synth.pair_labels(s, 4, "class") for s in specs]
    params = [gcvo.params_from_spec(specs[0], **ISO), gcvo.params_from_spec(specs[1], max_iters=300)]
    note("register_batch_labeled isotropic + anisotropic")
    tgt = np.concatenate([s.target for s in specs])
    src = np.concatenate([s.source for s in specs])
    to = np.cumsum([0] + [len(s.target) for s in specs])
    so = np.cumsum([0] + [len(s.source) for s in specs])
    LX = np.concatenate([lab[0] for lab in labels])
    LZ = np.concatenate([lab[1] for lab in labels])
    T, infos = gcvo.gcvo_register_batch_labeled(to_dev(tgt), to_dev(LX), to, to_dev(src), to_dev(LZ), so, None,
                                                params)
    refs = [O.register_spec(specs[0], LX=_f64(labels[0][0]), LZ=_f64(labels[0][1]), **ISO),
            O.register_spec(specs[1], LX=_f64(labels[1][0]), LZ=_f64(labels[1][1]), max_iters=300)]
    for k in range(2):
        dr, dt = rot_err_deg(T[k], refs[k].T), trans_err_m(T[k], refs[k].T)
        note(f"  pair {k}: iters {infos[k]['iters']} (oracle {refs[k].iters}) err {dr:.2e} deg {dt:.2e} m")
        assert refs[k].converged and infos[k]["converged"]
        assert dr < ROT_GATE_DEG and dt < TRANS_GATE_M
    s = specs[0]
    T1, i1 = gcvo.gcvo_register_batch_labeled(to_dev(s.target), to_dev(labels[0][0]), [0, len(s.target)],
                                              to_dev(s.source), to_dev(labels[0][1]), [0, len(s.source)], None,
                                              params[0])
    dr, dt = rot_err_deg(T1[0], refs[0].T), trans_err_m(T1[0], refs[0].T)
    note(f"  isotropic kernel alone: iters {i1[0]['iters']} err {dr:.2e} deg {dt:.2e} m")
    assert i1[0]["converged"] and dr < ROT_GATE_DEG and dt < TRANS_GATE_M
