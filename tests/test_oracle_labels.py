"""Pins of the oracle's label weights c_ij = <l^X_i, l^Z_j> (eq. rkhs_loss) and
of the isotropic special case (Remark 3), no GPU.

Independent facts: with one-hot class labels the weighted sums split exactly
into per-class unweighted sums; scaling the labels scales f, g and H alike and
leaves the Gauss-Newton step unchanged; the weighted gradient matches central
differences of the weighted objective; unit labels change nothing.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_10019_amd import synth


@pytest.fixture(scope="module")
def cloud():
    spec = synth.make_config1(2, n=500)
    X, Z = spec.target.astype(np.float64), spec.source.astype(np.float64)
    SX, SZ = O.point_shapes(X, 10, 0.05), O.point_shapes(Z, 10, 0.05)
    rng = np.random.default_rng(8)
    T = O.se3_exp(rng.normal(size=6) * 0.03)
    return X, SX, Z, SZ, T, rng


def test_unit_labels_change_nothing(cloud):
    X, SX, Z, SZ, T, _ = cloud
    a = O.evaluate(X, SX, Z, SZ, T, 0.3, 0.9)
    b = O.evaluate(X, SX, Z, SZ, T, 0.3, 0.9, LX=np.ones(len(X)), LZ=np.ones(len(Z)))
    assert a.f == b.f and np.array_equal(a.g, b.g) and np.array_equal(a.Hmain, b.Hmain) and a.npairs == b.npairs


def test_one_hot_labels_split_into_classes(cloud):
    X, SX, Z, SZ, T, rng = cloud
    cx, cz = rng.integers(0, 3, size=len(X)), rng.integers(0, 3, size=len(Z))
    e = O.evaluate(X, SX, Z, SZ, T, 0.3, 0.9, LX=np.eye(3)[cx], LZ=np.eye(3)[cz], with_t=True)
    f = 0.0
    g = np.zeros(6)
    H = np.zeros((6, 6))
    T1 = np.zeros((6, 6))
    for c in range(3):
        s = O.evaluate(X[cx == c], SX[cx == c], Z[cz == c], SZ[cz == c], T, 0.3, 0.9, with_t=True)
        f, g, H, T1 = f + s.f, g + s.g, H + s.Hmain, T1 + s.T1
    assert abs(e.f - f) <= 1e-12 * f
    np.testing.assert_allclose(e.g, g, rtol=0, atol=1e-11 * np.abs(g).max())
    np.testing.assert_allclose(e.Hmain, H, rtol=0, atol=1e-11 * np.abs(H).max())
    np.testing.assert_allclose(e.T1, T1, rtol=0, atol=1e-11 * np.abs(T1).max())


def test_label_scaling(cloud):
    X, SX, Z, SZ, T, rng = cloud
    LX, LZ = rng.uniform(0.5, 1.5, size=(len(X), 2)), rng.uniform(0.5, 1.5, size=(len(Z), 2))
    a = O.evaluate(X, SX, Z, SZ, T, 0.3, 0.9, LX=LX, LZ=LZ)
    b = O.evaluate(X, SX, Z, SZ, T, 0.3, 0.9, LX=2.0 * LX, LZ=3.0 * LZ)
    assert abs(b.f - 6.0 * a.f) <= 1e-12 * b.f
    np.testing.assert_allclose(b.g, 6.0 * a.g, rtol=1e-12, atol=1e-12 * np.abs(b.g).max())
    xa, _ = O.solve_step(a.H_gn, a.Hmain, a.g)
    xb, _ = O.solve_step(b.H_gn, b.Hmain, b.g)
    np.testing.assert_allclose(xa, xb, rtol=1e-10, atol=1e-14)


def test_labelled_gradient_matches_central_differences(cloud):
    X, SX, Z, SZ, T, rng = cloud
    LX, LZ = rng.uniform(0.0, 1.0, size=(len(X), 3)), rng.uniform(0.0, 1.0, size=(len(Z), 3))
    e = O.evaluate(X, SX, Z, SZ, T, 0.4, None, LX=LX, LZ=LZ)
    h = 1e-6
    fd = np.zeros(6)
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        fp = O.evaluate(X, SX, Z, SZ, T @ O.se3_exp(d), 0.4, None, R_shape=T[:3, :3], LX=LX, LZ=LZ).f
        fm = O.evaluate(X, SX, Z, SZ, T @ O.se3_exp(-d), 0.4, None, R_shape=T[:3, :3], LX=LX, LZ=LZ).f
        fd[k] = (fp - fm) / (2 * h)
    np.testing.assert_allclose(e.g, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())


def test_isotropic_shapes_are_the_identity():
    """rho = 1 floors every eigenvalue ratio at 1: S = U I U^T = I (Remark 3)."""
    spec = synth.make_config1(1, n=300)
    S = O.point_shapes(spec.target.astype(np.float64), 10, 1.0)
    np.testing.assert_allclose(S, np.tile([1.0, 0, 0, 1.0, 0, 1.0], (300, 1)), atol=1e-14)
