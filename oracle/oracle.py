"""ctypes wrapper of the FP64 CPU oracle (``liboracle_gcvo.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

All arrays are float64 numpy arrays; clouds are ``[n, 3]``, shapes ``[n, 6]``
in (xx, xy, xz, yy, yz, zz) order, poses 4x4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gcvo_oracle.c")
LIB = os.path.join(HERE, "liboracle_gcvo.so")

OK, ERR_INVALID, ERR_TOO_FEW_POINTS, ERR_NO_PAIRS, ERR_SINGULAR = 0, -1, -2, -3, -4

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_llp = ctypes.POINTER(ctypes.c_longlong)
_ip = ctypes.POINTER(ctypes.c_int)


CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def compile_to(src: str, out: str, extra=()) -> str:
    """gcc build of an oracle source file into the shared library ``out``."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP on)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    return LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = load(LIB)
    return _lib


def load(path: str) -> ctypes.CDLL:
    """Open an oracle build at ``path`` with the argument types declared (the
    tests also open builds of deliberately altered copies of the source)."""
    L = ctypes.CDLL(path)
    L.orc_knn.argtypes = [_dp, ctypes.c_long, ctypes.c_int, _lp]
    L.orc_point_shapes.argtypes = [_dp, ctypes.c_long, ctypes.c_int, ctypes.c_double, _dp]
    L.orc_eval.argtypes = [_dp, _dp, ctypes.c_long, _dp, _dp, ctypes.c_long, _dp, _dp,
                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                           _dp, _dp, _dp, _dp, _dp, _llp]
    L.orc_connection.argtypes = [_dp, _dp]
    L.orc_connection.restype = None
    L.orc_se3_exp.argtypes = [_dp, _dp]
    L.orc_se3_exp.restype = None
    L.orc_solve_step.argtypes = [_dp, _dp, _dp, _dp, _ip]
    L.orc_register.argtypes = [_dp, _dp, ctypes.c_long, _dp, _dp, ctypes.c_long, _dp,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_double, _dp, _dp]
    L.orc_line_coeffs.argtypes = [_dp, _dp, ctypes.c_long, _dp, _dp, ctypes.c_long, _dp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _dp, _dp, _llp]
    L.orc_first_order_step.argtypes = [_dp, ctypes.c_double, _dp]
    L.orc_eval_l.argtypes = [_dp, _dp, _dp, ctypes.c_long, _dp, _dp, _dp, ctypes.c_long, ctypes.c_int, _dp, _dp,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _llp]
    L.orc_register_l.argtypes = [_dp, _dp, _dp, ctypes.c_long, _dp, _dp, _dp, ctypes.c_long, ctypes.c_int, _dp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, _dp, _dp]
    L.orc_num_threads.argtypes = []
    L.orc_set_grid_threshold.argtypes = [ctypes.c_longlong]
    L.orc_set_grid_threshold.restype = None
    return L


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray | None):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def num_threads() -> int:
    return int(lib().orc_num_threads())


GRID_DEFAULT_MIN_PAIRS = 25_000_000


def set_grid_threshold(min_pairs: int) -> None:
    """Pair search of the sums: a uniform grid when nx * nz >= min_pairs (and
    there is a cutoff), else brute force.  Both give the same index lists, so
    the same results bit for bit; 0 forces the grid, a huge value brute force."""
    lib().orc_set_grid_threshold(int(min_pairs))


def knn(P, k: int) -> np.ndarray:
    P = _d(P)
    out = np.zeros((len(P), k), dtype=np.int64)
    st = lib().orc_knn(_p(P), len(P), k, out.ctypes.data_as(_lp))
    if st:
        raise OracleError(st, "orc_knn")
    return out


def point_shapes(P, k: int = 10, rho: float = 0.01) -> np.ndarray:
    P = _d(P)
    S = np.zeros((len(P), 6))
    st = lib().orc_point_shapes(_p(P), len(P), k, float(rho), _p(S))
    if st:
        raise OracleError(st, "orc_point_shapes")
    return S


@dataclass
class Eval:
    f: float
    g: np.ndarray
    Hmain: np.ndarray
    T1: np.ndarray | None
    T2: np.ndarray | None
    npairs: int

    @property
    def H_gn(self) -> np.ndarray:
        return self.Hmain + connection(self.g)


def _labels(LX, LZ, nx, nz):
    if LX is None and LZ is None:
        return None, None, 0
    LX, LZ = _d(LX), _d(LZ)
    LX = LX.reshape(nx, -1)
    LZ = LZ.reshape(nz, -1)
    if LX.shape[1] != LZ.shape[1]:
        raise ValueError("label dimensions differ")
    return np.ascontiguousarray(LX), np.ascontiguousarray(LZ), LX.shape[1]


def evaluate(X, SX, Z, SZ, T, ell: float, cutoff: float | None, sigma2: float = 1.0,
             R_shape=None, with_t: bool = False, LX=None, LZ=None) -> Eval:
    """f, g, H_main (and T1, T2) at T; LX, LZ: optional per-point label vectors
    [n, d] whose inner products weight the pairs."""
    X, SX, Z, SZ, T = _d(X), _d(SX), _d(Z), _d(SZ), _d(T)
    LX, LZ, dim = _labels(LX, LZ, len(X), len(Z))
    Rs = None if R_shape is None else _d(R_shape)
    f = ctypes.c_double()
    g = np.zeros(6)
    H = np.zeros((6, 6))
    T1 = np.zeros((6, 6)) if with_t else None
    T2 = np.zeros((6, 6)) if with_t else None
    npairs = ctypes.c_longlong()
    st = lib().orc_eval_l(_p(X), _p(SX), _p(LX), len(X), _p(Z), _p(SZ), _p(LZ), len(Z), dim, _p(T), _p(Rs),
                          float(ell), float(cutoff) if cutoff is not None else -1.0, float(sigma2),
                          ctypes.byref(f), _p(g), _p(H), _p(T1), _p(T2), ctypes.byref(npairs))
    if st:
        raise OracleError(st, "orc_eval")
    return Eval(f.value, g, H, T1, T2, npairs.value)


def line_coeffs(X, SX, Z, SZ, T, xi, ell: float, cutoff: float | None, sigma2: float = 1.0):
    """(c[0..4], npairs): G(t) = f(T exp(t xi^)) ~ sum_k c[k] t^k with the
    covariances frozen at T."""
    X, SX, Z, SZ, T, xi = _d(X), _d(SX), _d(Z), _d(SZ), _d(T), _d(xi)
    c = np.zeros(5)
    npairs = ctypes.c_longlong()
    st = lib().orc_line_coeffs(_p(X), _p(SX), len(X), _p(Z), _p(SZ), len(Z), _p(T), float(ell),
                               float(cutoff) if cutoff is not None else -1.0, float(sigma2), _p(xi), _p(c),
                               ctypes.byref(npairs))
    if st:
        raise OracleError(st, "orc_line_coeffs")
    return c, npairs.value


def first_order_step(c, min_step: float):
    """(mu, kind): kind 1 = smallest positive root of G' (mu = max(min_step,
    root)), 2 = quadratic-model step, 0 = min_step."""
    c = _d(c)
    mu = ctypes.c_double()
    kind = lib().orc_first_order_step(_p(c), float(min_step), ctypes.byref(mu))
    return mu.value, int(kind)


def connection(g) -> np.ndarray:
    g = _d(g)
    C = np.zeros((6, 6))
    lib().orc_connection(_p(g), _p(C))
    return C


def se3_exp(xi) -> np.ndarray:
    xi = _d(xi)
    T = np.zeros((4, 4))
    lib().orc_se3_exp(_p(xi), _p(T))
    return T


def solve_step(H, Hmain, g):
    H, Hmain, g = _d(H), _d(Hmain), _d(g)
    xi = np.zeros(6)
    damped = ctypes.c_int()
    st = lib().orc_solve_step(_p(H), _p(Hmain), _p(g), _p(xi), ctypes.byref(damped))
    if st:
        raise OracleError(st, "orc_solve_step")
    return xi, damped.value


@dataclass
class RegResult:
    T: np.ndarray
    converged: bool
    iters: int
    stages: int
    f: float
    g: np.ndarray
    xi_l1: float
    pairs_last: int
    damped_steps: int
    stage_iters: list


def register(X, Z, T_init=None, *, SX=None, SZ=None, length_scale: float, length_scale_min=None,
             anneal_factor: float = 0.5, cutoff_scale: float = 3.0, knn: int = 10,
             eig_ratio_min: float = 0.01, sigma2: float = 1.0, max_iters: int = 30,
             max_iters_per_stage: int = 30, tol: float = 1e-6, stage_tol: float = 1e-4,
             newton: bool = False, solver: int | None = None, min_step: float = 1e-10, LX=None,
             LZ=None) -> RegResult:
    """solver: 0 Gauss-Newton, 1 exact frozen-covariance Hessian (newton=True),
    2 first-order ascent with the quartic line search.  LX, LZ: optional
    per-point label vectors weighting the pairs."""
    solver = (1 if newton else 0) if solver is None else int(solver)
    X, Z = _d(X), _d(Z)
    T0 = np.eye(4) if T_init is None else _d(T_init)
    lmin = length_scale if length_scale_min is None else length_scale_min
    SXp = None if SX is None else _d(SX)
    SZp = None if SZ is None else _d(SZ)
    Tout = np.zeros((4, 4))
    info = np.zeros(32)
    LXp, LZp, dim = _labels(LX, LZ, len(X), len(Z))
    st = lib().orc_register_l(_p(X), _p(SXp), _p(LXp), len(X), _p(Z), _p(SZp), _p(LZp), len(Z), dim, _p(T0),
                            float(length_scale), float(lmin), float(anneal_factor), float(cutoff_scale),
                            int(knn), float(eig_ratio_min), float(sigma2), int(max_iters),
                            int(max_iters_per_stage), float(tol), float(stage_tol), solver, float(min_step),
                            _p(Tout), _p(info))
    if st:
        raise OracleError(st, "orc_register")
    nst = int(info[3])
    return RegResult(T=Tout, converged=bool(info[1]), iters=int(info[2]), stages=nst, f=float(info[4]),
                     g=info[5:11].copy(), xi_l1=float(info[11]), pairs_last=int(info[12]),
                     damped_steps=int(info[13]), stage_iters=[int(v) for v in info[14:14 + min(nst, 16)]])


def register_spec(spec, T_init=None, SX=None, SZ=None, **overrides) -> RegResult:
    """Register a ``synth.PairSpec`` with its own solver settings (overridable)."""
    p = spec.params()
    p.update(overrides)
    return register(spec.target.astype(np.float64), spec.source.astype(np.float64), T_init,
                    SX=SX, SZ=SZ, **p)
