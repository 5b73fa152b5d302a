"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and its host-side sizing/validation functions behave (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_2606_10019_amd import gcvo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gcvo_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gcvo.load_library()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(gcvo.EXPORTED)


def test_struct_layouts_match_header():
    # sizes implied by the header's field order on x86-64
    assert ctypes.sizeof(gcvo.gcvo_params) == 8 * 4 + 8 + 8 * 2 + 8 + 8 * 2 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(gcvo.gcvo_info) == 4 * 4 + 8 + 8 + 48 + 8 + 4 * 16 + 4 + 4   # damped, then padding
    assert ctypes.sizeof(gcvo.gcvo_profile) == 8 * 4
    assert gcvo.load_library().gcvo_abi_version() == 200
    assert not gcvo.default_params().profile          # no measurement unless asked for


def test_default_params_and_strerror():
    p = gcvo.default_params()
    assert p.length_scale == 0.3 and p.knn == 10 and p.cutoff_scale == 3.0 and p.max_iters == 30
    for code in range(-7, 1):
        assert gcvo.strerror(code)
    assert "unknown" in gcvo.strerror(-99)


def test_workspace_size_validation():
    p = gcvo.default_params()
    a = gcvo.gcvo_workspace_size(2000, 2000, p)
    b = gcvo.gcvo_workspace_size(20000, 20000, p)
    assert 0 < a < b
    assert gcvo.gcvo_workspace_size(0, 10, p) == 0
    bad = gcvo.default_params(knn=1)
    assert gcvo.gcvo_workspace_size(100, 100, bad) == 0
    bad = gcvo.default_params(length_scale_min=0.5)   # min above start
    assert gcvo.gcvo_workspace_size(100, 100, bad) == 0
    bad = gcvo.default_params(length_scale=1.0, length_scale_min=0.1, anneal_factor=1.0)
    assert gcvo.gcvo_workspace_size(100, 100, bad) == 0
    assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(solver=3)) == 0
    assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(solver=2, min_step=0.0)) == 0
    assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(solver=2)) > 0
    for cf in (0.1, 1.5, float("nan")):
        assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(cell_fraction=cf)) == 0
    assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(cell_fraction=0.25)) > 0
    for cf in (0.05, 1.5):
        assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(cell_fraction_x=cf)) == 0
    assert gcvo.gcvo_workspace_size(100, 100, gcvo.default_params(cell_fraction_x=0.125)) > 0
    # annealing 1.0 -> 0.1 by halves: 5 stages need more space than one stage
    ann = gcvo.default_params(length_scale=1.0, length_scale_min=0.1, anneal_factor=0.5)
    assert gcvo.gcvo_workspace_size(2000, 2000, ann) > gcvo.gcvo_workspace_size(2000, 2000, gcvo.default_params(
        length_scale=1.0, length_scale_min=1.0))
    assert gcvo.load_library().gcvo_eval_workspace_size(100, 100) > 0
    assert gcvo.load_library().gcvo_shapes_workspace_size(100) > 0
    assert gcvo.load_library().gcvo_shapes_workspace_size(0) == 0


def test_batch_workspace_covers_members():
    import numpy as np
    p = gcvo.default_params()
    off = np.array([0, 1000, 3000, 3500], dtype=np.int64)
    whole = gcvo.gcvo_batch_workspace_size(off, off, p)
    assert whole > gcvo.gcvo_workspace_size(2000, 2000, p)
    # pairs too small to run still get an output slot: the size is positive
    tiny = np.array([0, 3, 5], dtype=np.int64)
    assert gcvo.gcvo_batch_workspace_size(tiny, tiny, p) > 0


def test_batched_shapes_and_eval_sizes_and_validation():
    import numpy as np
    L = gcvo.load_library()
    off = np.array([0, 1000, 3000], dtype=np.int64)
    op = off.ctypes.data_as(ctypes.c_void_p)
    one = np.array([0, 2000], dtype=np.int64)
    assert L.gcvo_shapes_batch_workspace_size(2, op) > L.gcvo_shapes_workspace_size(2000)
    assert L.gcvo_shapes_batch_workspace_size(0, op) == 0
    assert L.gcvo_shapes_batch_workspace_size(2, None) == 0
    assert L.gcvo_eval_batch_workspace_size(2, op, op) > 0
    assert L.gcvo_eval_batch_workspace_size(1, one.ctypes.data_as(ctypes.c_void_p), None) == 0
    # a cloud with fewer points than knn is refused before any device work
    small = np.array([0, 1000, 1005], dtype=np.int64)
    st = L.gcvo_point_shapes_batch(2, ctypes.c_void_p(16), small.ctypes.data_as(ctypes.c_void_p), 10, 0.1,
                                   ctypes.c_void_p(16), None, 0, None)
    assert st == gcvo.GCVO_ERR_TOO_FEW_POINTS
    ell = np.array([0.3, -1.0])
    st = L.gcvo_eval_fgh_batch(2, ctypes.c_void_p(16), ctypes.c_void_p(16), op, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), op, None, ell.ctypes.data_as(ctypes.c_void_p), 3.0, 1.0, 0,
                               None, None, None, None, None, None, 0, None)
    assert st == gcvo.GCVO_ERR_INVALID                # a non-positive length scale


def test_register_rejects_bad_arguments_without_gpu_work():
    L = gcvo.load_library()
    p = gcvo.default_params()
    T = (ctypes.c_double * 16)()
    info = gcvo.gcvo_info()
    # null clouds
    st = L.gcvo_register(None, 100, None, 100, None, ctypes.byref(p), T, ctypes.byref(info), None, 0, None)
    assert st == gcvo.GCVO_ERR_INVALID and info.status == st
    # a non-rigid initial pose is rejected before anything is enqueued
    bad = (ctypes.c_double * 16)(*([2.0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1]))
    st = L.gcvo_register(ctypes.c_void_p(16), 100, ctypes.c_void_p(16), 100, bad, ctypes.byref(p), T,
                         ctypes.byref(info), None, 0, None)
    assert st == gcvo.GCVO_ERR_INVALID
    # too few points for knn
    st = L.gcvo_register(ctypes.c_void_p(16), 5, ctypes.c_void_p(16), 100, None, ctypes.byref(p), T,
                         ctypes.byref(info), None, 0, None)
    assert st == gcvo.GCVO_ERR_TOO_FEW_POINTS
    # a cloud beyond GCVO_MAX_POINTS (2^26) is refused before its memory is touched
    st = L.gcvo_register(ctypes.c_void_p(16), (1 << 26) + 1, ctypes.c_void_p(16), 100, None, ctypes.byref(p), T,
                         ctypes.byref(info), None, 0, None)
    assert st == gcvo.GCVO_ERR_CAPACITY and info.status == st
    assert gcvo.gcvo_workspace_size((1 << 26) + 1, 100, p) == 0
    assert all(v == 0.0 for v in T)   # pose output untouched


def test_mlp_sizes():
    L = gcvo.load_library()
    assert L.gcvo_mlp_param_count() == gcvo.GCVO_MLP_N_PARAMS == 42246
    assert ctypes.sizeof(gcvo.gcvo_mlp_batch) == 4 + 4 + 8 * 4 + 8 * 4 + 8 * 4 + 8
    a = gcvo.gcvo_mlp_workspace_size(16, 1024)
    assert 0 < a < gcvo.gcvo_mlp_workspace_size(128, 1024)
    assert gcvo.gcvo_mlp_workspace_size(0, 1024) == 0
    assert gcvo.gcvo_mlp_workspace_size(4, 0) == 0
    assert gcvo.gcvo_mlp_workspace_size(4, 1 << 20) == 0


def test_labeled_and_isotropic_sizes_and_validation():
    import numpy as np
    L = gcvo.load_library()
    p = gcvo.default_params()
    off = np.array([0, 2000], dtype=np.int64)
    plain = gcvo.gcvo_batch_workspace_size(off, off, p)
    lab = gcvo.gcvo_batch_workspace_size_labeled(off, off, p, 3)
    assert lab > plain                       # label rows per source point and per stage
    assert gcvo.gcvo_batch_workspace_size_labeled(off, off, p, 0) == 0
    assert gcvo.gcvo_batch_workspace_size_labeled(off, off, p, gcvo.GCVO_MAX_LABEL_DIM + 1) == 0
    # rho = 1: no neighbourhoods, so no kNN grids or shape arrays
    iso = gcvo.default_params(eig_ratio_min=1.0)
    assert 0 < gcvo.gcvo_workspace_size(2000, 2000, iso) < gcvo.gcvo_workspace_size(2000, 2000, p)
    assert L.gcvo_eval_workspace_size_labeled(100, 100, 2) > L.gcvo_eval_workspace_size(100, 100)
    assert L.gcvo_eval_workspace_size_labeled(100, 100, 5) == 0
    op = off.ctypes.data_as(ctypes.c_void_p)
    # labelled calls without labels, or with a bad width, fail before any device work
    # (the pose and info outputs are device pointers the call never touches here)
    for dim, tl in ((2, None), (0, 16), (5, 16)):
        st = L.gcvo_register_batch_labeled(1, ctypes.c_void_p(16), tl, op, ctypes.c_void_p(16), tl, op, dim, None,
                                           ctypes.byref(p), 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0,
                                           None)
        assert st == gcvo.GCVO_ERR_INVALID, dim
    f = ctypes.c_double()
    g = np.zeros(6)
    H = np.zeros(36)
    I = np.eye(4).ravel()
    st = L.gcvo_eval_fgh_labeled(ctypes.c_void_p(16), ctypes.c_void_p(16), None, 10, ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), None, 10, 2, I.ctypes.data_as(ctypes.c_void_p), 0.5, 1.5, 1.0,
                                 0, ctypes.byref(f), g.ctypes.data_as(ctypes.c_void_p),
                                 H.ctypes.data_as(ctypes.c_void_p), None, None, 0, None)
    assert st == gcvo.GCVO_ERR_INVALID


def test_autotune_candidates_copy_parameters():
    from paper_2606_10019_amd import autotune
    p = gcvo.default_params(length_scale=0.7, knn=12)
    q = autotune._with_fraction(p, (0.7, 0.125))
    assert (q.cell_fraction, q.cell_fraction_x) == (0.7, 0.125)
    assert (q.length_scale, q.knn) == (0.7, 12)
    assert (p.cell_fraction, p.cell_fraction_x) == (0.5, 0.125)    # the caller's set is untouched
    qs = autotune._with_fraction([p, p], 0.35)
    assert [(x.cell_fraction, x.cell_fraction_x) for x in qs] == [(0.35, 0.35)] * 2
    for cand in autotune.CANDIDATES:                                # every candidate is a valid parameter set
        assert gcvo.gcvo_workspace_size(500, 500, autotune._with_fraction(p, cand)) > 0
