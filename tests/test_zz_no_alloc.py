"""The evaluation entry point that allocates nothing (gcvo_eval_fgh_noalloc)
against the workspace one (gcvo_eval_fgh), through the C ABI (run on an
MI355X).

Both run the same kernels on the same inputs, so the results must be bitwise
equal.  Two calls in a row, the second with a smaller input, check that the
shared per-GPU scratch holds nothing one call depends on from the previous one.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2606_10019_amd import gcvo, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.device("cuda:0"))


def note(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("precision", [gcvo.GCVO_PRECISION_FP32, gcvo.GCVO_PRECISION_FP64])
def test_noalloc_eval_equals_workspace_eval(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spec = synth.make_config1(0)
    SX = O.point_shapes(spec.target.astype(np.float64), 10, spec.eig_ratio_min).astype(np.float32)
    SZ = O.point_shapes(spec.source.astype(np.float64), 10, spec.eig_ratio_min).astype(np.float32)
    T = np.eye(4)
    T[:3, 3] = [0.05, -0.03, 0.02]
    # a full-size call, then a smaller one (a prefix of both clouds)
    for nt, ns in ((len(spec.target), len(spec.source)), (700, 513)):
        tx, ts = to_dev(spec.target[:nt]), to_dev(SX[:nt].T)
        sx, ss = to_dev(spec.source[:ns]), to_dev(SZ[:ns].T)
        note(f"noalloc eval {nt} / {ns} points, precision {precision}")
        a = gcvo.gcvo_eval_fgh_noalloc(tx, ts, sx, ss, T, 0.3, 0.9, 1.0, precision)
        b = gcvo.gcvo_eval_fgh(tx, ts, sx, ss, T, 0.3, 0.9, 1.0, precision)
        note(f"  f {a.f:.12g} vs {b.f:.12g}, pairs {a.npairs} vs {b.npairs}")
        assert a.npairs == b.npairs > 0
        assert a.f == b.f and np.array_equal(a.g, b.g) and np.array_equal(a.H, b.H)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    L = gcvo.load_library()
    n = 400_000                                   # needs about 105 MiB of scratch
    assert L.gcvo_eval_workspace_size(n, n) > gcvo.GCVO_NOALLOC_SCRATCH_BYTES
    f = ctypes.c_double()
    g = np.zeros(6)
    H = np.zeros(36)
    I = np.eye(4).ravel()
    st = L.gcvo_eval_fgh_noalloc(ctypes.c_void_p(16), ctypes.c_void_p(16), n, ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), n, I.ctypes.data_as(ctypes.c_void_p), 0.3, 0.9, 1.0, 0,
                                 ctypes.byref(f), g.ctypes.data_as(ctypes.c_void_p),
                                 H.ctypes.data_as(ctypes.c_void_p), None, None)
    assert st == gcvo.GCVO_ERR_CAPACITY
