"""The damped branch of the Gauss-Newton step and its failure on the GPU,
against the FP64 oracle (run on an MI355X).

The step of eq. (gn_update) solves H_GN xi = -g.  Reading of the damping the
paper leaves open (both sides): when that step is not an ascent direction or
H_GN is numerically singular, the connection term is dropped and
(H_main - lambda ||diag H_main||_2 I) xi = -g is solved for lambda = 1e-6 *
10^m, m = 0..6; when none of these gives an ascent direction the pair fails
with GCVO_ERR_SINGULAR.

Inputs that reach these branches come from the labelled objective of eq.
(rkhs_loss), whose weights c_ij = <l^X_i, l^Z_j> may be negative:
  * every target label -1: f < 0 and H_main is positive semi-definite, so the
    plain step descends and the damped shift loop supplies the step;
  * two targets at +r and -r from one source point with labels +1 and -1: the
    two pair terms of f and H_main cancel exactly while those of g add, so
    H_main = 0 with g != 0, and no damped system can be solved.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2606_10019_amd import gcvo, synth  # noqa: E402
from tests.posemetrics import rot_err_deg, trans_err_m  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def register_labeled(X, Z, LX, LZ, **kw):
    p = gcvo.default_params(**kw)
    T, infos = gcvo.gcvo_register_batch_labeled(to_dev(X), to_dev(LX), [0, len(X)], to_dev(Z), to_dev(LZ),
                                                [0, len(Z)], None, p)
    return T[0], infos[0]


def negative_problem():
    spec = synth.make_config1(0, n=800)
    X, Z = spec.target, spec.source
    return X, Z, np.full((len(X), 1), -1.0, np.float32), np.ones((len(Z), 1), np.float32)


@pytest.mark.parametrize("precision", [gcvo.GCVO_PRECISION_FP64, gcvo.GCVO_PRECISION_FP32])
def test_damped_step_matches_oracle(precision):
    X, Z, LX, LZ = negative_problem()
    kw = dict(length_scale=0.3, length_scale_min=0.3, eig_ratio_min=0.01, max_iters=1, tol=1e-8)
    ref = O.register(X.astype(np.float64), Z.astype(np.float64), LX=LX.astype(np.float64), LZ=LZ.astype(np.float64),
                     **kw)
    note(f"damped step, all target labels -1, precision {precision}: oracle damped {ref.damped_steps}")
    assert ref.damped_steps == 1                     # the input does reach the damped branch
    T, info = register_labeled(X, Z, LX, LZ, precision=precision, **kw)
    dr, dt = rot_err_deg(T, ref.T), trans_err_m(T, ref.T)
    note(f"  GPU status {info['status']} damped {info['damped']} iters {info['iters']}; pose vs oracle "
         f"{dr:.2e} deg {dt:.2e} m (step {np.linalg.norm(ref.T[:3, 3]):.3f} m)")
    assert info["status"] == gcvo.GCVO_OK and info["iters"] == 1 and info["damped"] == 1
    # The registration computes its own shapes, which the library stores in
    # float32 whatever the kernels' precision, so even the FP64 kernels see
    # shapes rounded to float32: the step agrees within the accuracy gate and
    # f within the FP32 bound of the shapes' rounding (64 eps32 / rho).
    assert dr < 1e-3 and dt < 1e-5
    assert abs(info["f"] - ref.f) <= 64 * float(np.finfo(np.float32).eps) / 0.01 * abs(ref.f)


def test_pushed_apart_pair_reports_no_pairs():
    """After the damped step the negative weights push the clouds beyond the
    cutoff: the next evaluation has no pair, on both sides."""
    X, Z, LX, LZ = negative_problem()
    kw = dict(length_scale=0.3, length_scale_min=0.3, eig_ratio_min=0.01, max_iters=3, tol=1e-8)
    with pytest.raises(O.OracleError) as e:
        O.register(X.astype(np.float64), Z.astype(np.float64), LX=LX.astype(np.float64), LZ=LZ.astype(np.float64),
                   **kw)
    assert e.value.status == O.ERR_NO_PAIRS
    T, info = register_labeled(X, Z, LX, LZ, precision=gcvo.GCVO_PRECISION_FP64, **kw)
    note(f"pushed apart: GPU status {info['status']} iters {info['iters']}")
    assert info["status"] == gcvo.GCVO_ERR_NO_PAIRS
    assert np.array_equal(T, np.eye(4))              # a failed pair keeps its start pose


def symmetric_signed_pair():
    X = np.array([[0.5, 0, 0], [-0.5, 0, 0]], np.float32)
    Z = np.array([[0, 0, 0], [0, 0, 10.0]], np.float32)
    return X, Z, np.array([[1.0], [-1.0]], np.float32), np.ones((2, 1), np.float32)


@pytest.mark.parametrize("precision", [gcvo.GCVO_PRECISION_FP32, gcvo.GCVO_PRECISION_FP64])
def test_zero_hessian_is_singular(precision):
    X, Z, LX, LZ = symmetric_signed_pair()
    X64, Z64 = X.astype(np.float64), Z.astype(np.float64)
    # shapes rounded to float32 on both sides (the library reads float32 shapes)
    SX = O.point_shapes(X64, 2, 0.1).astype(np.float32).astype(np.float64)
    SZ = O.point_shapes(Z64, 2, 0.1).astype(np.float32).astype(np.float64)
    o = O.evaluate(X64, SX, Z64, SZ, np.eye(4), 1.0, 3.0, LX=LX.astype(np.float64), LZ=LZ.astype(np.float64))
    assert o.npairs == 2 and o.f == 0.0 and np.all(o.Hmain == 0.0) and np.abs(o.g).max() > 1.0
    e = gcvo.gcvo_eval_fgh_labeled(to_dev(X), to_dev(SX.T), to_dev(LX), to_dev(Z), to_dev(SZ.T), to_dev(LZ),
                                   np.eye(4), 1.0, 3.0, 1.0, precision)
    note(f"zero H_main, precision {precision}: GPU f {e.f} |g| {np.abs(e.g).max():.4f} (oracle "
         f"{np.abs(o.g).max():.4f}) H_GN - C(g) max {np.abs(e.H - O.connection(e.g)).max():.2e}")
    assert e.npairs == 2 and e.f == 0.0
    np.testing.assert_allclose(e.g, o.g, rtol=1e-6 if precision == gcvo.GCVO_PRECISION_FP32 else 1e-12, atol=0)
    assert np.all(e.H - O.connection(e.g) == 0.0)    # H_GN is the connection term alone
    with pytest.raises(O.OracleError) as ex:
        O.register(X64, Z64, length_scale=1.0, knn=2, eig_ratio_min=0.1, max_iters=5, LX=LX.astype(np.float64),
                   LZ=LZ.astype(np.float64))
    assert ex.value.status == O.ERR_SINGULAR
    # a start pose other than the identity, to see it kept (a shift along z
    # keeps the two pairs mirror images, so H_main stays exactly zero)
    T0 = np.eye(4)
    T0[2, 3] = 1e-3
    p = gcvo.default_params(length_scale=1.0, length_scale_min=1.0, knn=2, eig_ratio_min=0.1, max_iters=5,
                            precision=precision)
    T, infos = gcvo.gcvo_register_batch_labeled(to_dev(X), to_dev(LX), [0, 2], to_dev(Z), to_dev(LZ), [0, 2], T0[None],
                                                p)
    note(f"  GPU register: status {infos[0]['status']}")
    assert infos[0]["status"] == gcvo.GCVO_ERR_SINGULAR
    assert np.array_equal(T[0], T0)
