"""Pins of the oracle's solver variants (no GPU): the exact-Hessian (Newton)
solver and the first-order ascent with the quartic line search.

The line-search polynomial is pinned to quantities pinned elsewhere: its linear
coefficient is g . xi (Lemma 1), its quadratic coefficient is half of
xi^T D(g) xi with D(g) = T1 + T2 + H_main (pinned by finite differences), and
it matches the directly evaluated objective along the curve to fifth order.
The root finder is checked against numpy's polynomial roots, and both variants
must reach the Gauss-Newton fixed point (the zero of the same gradient).
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_10019_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_poses.json")))


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(21)
    spec = synth.make_config1(3, n=300)
    X, Z = spec.target.astype(np.float64), spec.source.astype(np.float64)
    SX, SZ = O.point_shapes(X, 10, 0.05), O.point_shapes(Z, 10, 0.05)
    T = O.se3_exp(rng.normal(size=6) * 0.05)
    return X, SX, Z, SZ, T, rng


def test_line_coefficients_match_gradient_and_exact_hessian(small):
    X, SX, Z, SZ, T, rng = small
    e = O.evaluate(X, SX, Z, SZ, T, 0.4, None, with_t=True)
    D = e.Hmain + e.T1 + e.T2
    for _ in range(3):
        xi = rng.normal(size=6) * np.array([0.1, 0.1, 0.1, 0.2, 0.2, 0.2])
        c, n = O.line_coeffs(X, SX, Z, SZ, T, xi, 0.4, None)
        assert n == e.npairs
        assert abs(c[0] - e.f) <= 1e-12 * e.f
        assert abs(c[1] - e.g @ xi) <= 1e-10 * np.abs(e.g) @ np.abs(xi)
        assert abs(2 * c[2] - xi @ D @ xi) <= 1e-9 * np.abs(xi) @ np.abs(D) @ np.abs(xi)


def test_quartic_matches_objective_to_fifth_order(small):
    X, SX, Z, SZ, T, rng = small
    xi = np.array([0.3, -0.2, 0.5, 0.4, 0.1, -0.3])
    c, _ = O.line_coeffs(X, SX, Z, SZ, T, xi, 0.4, None)

    def G(t):   # covariances frozen at T's rotation
        return O.evaluate(X, SX, Z, SZ, T @ O.se3_exp(t * xi), 0.4, None, R_shape=T[:3, :3]).f

    def err(t):
        return abs(G(t) - sum(c[k] * t ** k for k in range(5)))

    t = 0.02
    ratios = [err(t / 2 ** k) / err(t / 2 ** (k + 1)) for k in range(3)]
    assert all(22 < r < 45 for r in ratios), ratios          # 2^5 = 32: error is O(t^5)


def _smallest_positive_root(c):
    r = np.roots([4 * c[4], 3 * c[3], 2 * c[2], c[1]])
    real = [x.real for x in r if abs(x.imag) <= 1e-9 * max(1.0, abs(x))]
    pos = [x for x in real if x > 0]
    return min(pos) if pos else None


def test_step_root_matches_numpy_roots():
    rng = np.random.default_rng(4)
    checked = 0
    for k in range(3000):
        c = rng.normal(size=5) * 10.0 ** rng.integers(-3, 4, size=5)
        c[1] = abs(c[1]) + 1e-3                      # G'(0) = g . g > 0
        if k % 7 == 0:
            c[4] = 0.0
        if k % 11 == 0:
            c[3] = c[4] = 0.0
        mu, kind = O.first_order_step(c, 1e-300)
        ref = _smallest_positive_root(c)
        if kind == 1:
            assert ref is not None
            assert abs(mu - ref) <= 1e-9 * ref, (c, mu, ref)
            checked += 1
        elif kind == 2:
            assert ref is None and c[2] < 0
            assert mu == pytest.approx(c[1] / (-2 * c[2]), rel=1e-15)
        else:
            assert ref is None and c[2] >= 0 and mu == 1e-300
    assert checked > 1000


@pytest.mark.parametrize("solver", [1, 2])
def test_variants_reach_the_gauss_newton_fixed_point(solver):
    spec = synth.make_config1(0)
    ref = np.array(GOLDEN[spec.name]["T_ref"]).reshape(4, 4)
    r = O.register_spec(spec, solver=solver, tol=1e-10, max_iters=3000)
    assert r.converged
    assert np.max(np.abs(r.T - ref)) < 1e-7
    if solver == 1:
        assert r.iters < GOLDEN[spec.name]["ref_iters"]          # Newton: fewer iterations than GN
    else:
        assert r.iters > 10 * GOLDEN[spec.name]["prod_iters"]    # first order: much slower


def test_newton_from_identity_converges_where_pure_newton_diverges():
    """Config-1 instances where an unmodified Newton iteration from identity
    leaves the basin (indefinite exact Hessian far from the maximum): the
    switch to the Gauss-Newton system there keeps it on course."""
    for inst in (1, 2, 7):
        spec = synth.make_config1(inst)
        r = O.register_spec(spec, solver=1)
        ref = np.array(GOLDEN[spec.name]["T_ref"]).reshape(4, 4)
        assert r.converged and np.max(np.abs(r.T - ref)) < 1e-7, inst
