"""Python binding of the gfx950 G-CVO library (``libgcvo.so``).

Argument marshalling only: tensors are passed to the C ABI of
``include/gcvo.h`` as raw device pointers with the current HIP stream, and
every step of the computation runs in the library's kernels.  There is no CPU
fallback: if the library is missing or fails to load, every call raises.

Device tensors are torch CUDA (HIP) tensors: clouds float32 ``[n, 3]``
contiguous, shapes float32 ``[6, n]`` (xx, xy, xz, yy, yz, zz).  Single-pair
poses are float64 numpy ``4x4`` arrays on the host; the batch calls take and
give device poses (``[n, 4, 4]`` float64 tensors), with host numpy copies as
the default return for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcvo.so")

GCVO_OK = 0
GCVO_ERR_INVALID = -1
GCVO_ERR_TOO_FEW_POINTS = -2
GCVO_ERR_NO_PAIRS = -3
GCVO_ERR_SINGULAR = -4
GCVO_ERR_WORKSPACE = -5
GCVO_ERR_HIP = -6
GCVO_ERR_CAPACITY = -7
GCVO_PRECISION_FP32 = 0
GCVO_PRECISION_FP64 = 1
GCVO_SOLVER_GN = 0
GCVO_SOLVER_NEWTON = 1
GCVO_SOLVER_FIRST_ORDER = 2
GCVO_MAX_STAGES = 16
GCVO_MAX_LABEL_DIM = 4

EXPORTED = ["gcvo_default_params", "gcvo_workspace_size", "gcvo_register", "gcvo_batch_workspace_size",
            "gcvo_register_batch", "gcvo_eval_workspace_size", "gcvo_eval_fgh", "gcvo_shapes_workspace_size",
            "gcvo_point_shapes", "gcvo_strerror", "gcvo_abi_version",
            "gcvo_mlp_param_count", "gcvo_mlp_workspace_size", "gcvo_mlp_forward", "gcvo_mlp_loss_grad",
            "gcvo_mlp_adam", "gcvo_batch_workspace_size_labeled", "gcvo_register_batch_labeled",
            "gcvo_eval_workspace_size_labeled", "gcvo_eval_fgh_labeled", "gcvo_shapes_batch_workspace_size",
            "gcvo_point_shapes_batch", "gcvo_eval_batch_workspace_size", "gcvo_eval_fgh_batch",
            "gcvo_eval_fgh_noalloc"]
GCVO_NOALLOC_SCRATCH_BYTES = 64 << 20

GCVO_MLP_N_PARAMS = 42246
GCVO_MLP_ROT_SCALE = 0.3
GCVO_MLP_TRANS_SCALE = 3.0


class gcvo_profile(ctypes.Structure):
    _fields_ = [("pair_kernel_ms", ctypes.c_double), ("launches", ctypes.c_longlong),
                ("pairs", ctypes.c_longlong), ("source_points", ctypes.c_longlong)]

    def to_dict(self) -> dict:
        return dict(pair_kernel_ms=self.pair_kernel_ms, launches=self.launches, pairs=self.pairs,
                    source_points=self.source_points)


class gcvo_params(ctypes.Structure):
    _fields_ = [("length_scale", ctypes.c_double), ("length_scale_min", ctypes.c_double),
                ("anneal_factor", ctypes.c_double), ("cutoff_scale", ctypes.c_double),
                ("knn", ctypes.c_int), ("eig_ratio_min", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("max_iters", ctypes.c_int), ("max_iters_per_stage", ctypes.c_int),
                ("tol", ctypes.c_double), ("stage_tol", ctypes.c_double), ("precision", ctypes.c_int),
                ("solver", ctypes.c_int), ("min_step", ctypes.c_double), ("cell_fraction", ctypes.c_double),
                ("cell_fraction_x", ctypes.c_double), ("profile", ctypes.POINTER(gcvo_profile))]


class gcvo_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("converged", ctypes.c_int), ("iters", ctypes.c_int),
                ("stages", ctypes.c_int), ("pairs_last", ctypes.c_longlong), ("f", ctypes.c_double),
                ("g", ctypes.c_double * 6), ("xi_l1", ctypes.c_double),
                ("stage_iters", ctypes.c_int * GCVO_MAX_STAGES), ("damped", ctypes.c_int)]

    def to_dict(self) -> dict:
        return dict(status=self.status, converged=bool(self.converged), iters=self.iters, stages=self.stages,
                    pairs_last=self.pairs_last, f=self.f, g=list(self.g), xi_l1=self.xi_l1,
                    stage_iters=list(self.stage_iters)[:max(self.stages, 0)], damped=self.damped)


class gcvo_mlp_batch(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int), ("n_points", ctypes.c_int),
                ("tgt_xyz", ctypes.c_void_p), ("n_tgt_rows", ctypes.c_longlong),
                ("tgt_start", ctypes.c_void_p), ("tgt_count", ctypes.c_void_p),
                ("src_xyz", ctypes.c_void_p), ("n_src_rows", ctypes.c_longlong),
                ("src_start", ctypes.c_void_p), ("src_count", ctypes.c_void_p),
                ("tgt_idx", ctypes.c_void_p), ("src_idx", ctypes.c_void_p),
                ("tgt_motion", ctypes.c_void_p), ("src_motion", ctypes.c_void_p),
                ("input_scale", ctypes.c_float)]


class GcvoError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


_P = ctypes.c_void_p
_lib = None


def load_library() -> ctypes.CDLL:
    """Load libgcvo.so (built by ``__graft_entry__.build()``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the gfx950 library first (__graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(gcvo_params)
    L.gcvo_default_params.argtypes = [pp]
    L.gcvo_default_params.restype = None
    L.gcvo_workspace_size.argtypes = [ctypes.c_longlong, ctypes.c_longlong, pp]
    L.gcvo_workspace_size.restype = ctypes.c_size_t
    L.gcvo_register.argtypes = [_P, ctypes.c_longlong, _P, ctypes.c_longlong, _P, pp, _P,
                                ctypes.POINTER(gcvo_info), _P, ctypes.c_size_t, _P]
    L.gcvo_batch_workspace_size.argtypes = [ctypes.c_int, _P, _P, pp, ctypes.c_int]
    L.gcvo_batch_workspace_size.restype = ctypes.c_size_t
    L.gcvo_register_batch.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, pp, ctypes.c_int, _P, _P, _P,
                                      ctypes.c_size_t, _P]
    L.gcvo_eval_workspace_size.argtypes = [ctypes.c_longlong, ctypes.c_longlong]
    L.gcvo_eval_workspace_size.restype = ctypes.c_size_t
    L.gcvo_eval_fgh.argtypes = [_P, _P, ctypes.c_longlong, _P, _P, ctypes.c_longlong, _P, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P,
                                ctypes.c_size_t, _P]
    L.gcvo_batch_workspace_size_labeled.argtypes = [ctypes.c_int, _P, _P, pp, ctypes.c_int, ctypes.c_int]
    L.gcvo_batch_workspace_size_labeled.restype = ctypes.c_size_t
    L.gcvo_register_batch_labeled.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_int, _P, pp,
                                              ctypes.c_int, _P, _P, _P, ctypes.c_size_t, _P]
    L.gcvo_eval_workspace_size_labeled.argtypes = [ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int]
    L.gcvo_eval_workspace_size_labeled.restype = ctypes.c_size_t
    L.gcvo_eval_fgh_labeled.argtypes = [_P, _P, _P, ctypes.c_longlong, _P, _P, _P, ctypes.c_longlong, ctypes.c_int,
                                        _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P,
                                        _P, _P, _P, ctypes.c_size_t, _P]
    L.gcvo_shapes_workspace_size.argtypes = [ctypes.c_longlong]
    L.gcvo_shapes_workspace_size.restype = ctypes.c_size_t
    L.gcvo_point_shapes.argtypes = [_P, ctypes.c_longlong, ctypes.c_int, ctypes.c_double, _P, _P,
                                    ctypes.c_size_t, _P]
    L.gcvo_eval_fgh_noalloc.argtypes = [_P, _P, ctypes.c_longlong, _P, _P, ctypes.c_longlong, _P, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P]
    L.gcvo_shapes_batch_workspace_size.argtypes = [ctypes.c_int, _P]
    L.gcvo_shapes_batch_workspace_size.restype = ctypes.c_size_t
    L.gcvo_point_shapes_batch.argtypes = [ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_double, _P, _P,
                                          ctypes.c_size_t, _P]
    L.gcvo_eval_batch_workspace_size.argtypes = [ctypes.c_int, _P, _P]
    L.gcvo_eval_batch_workspace_size.restype = ctypes.c_size_t
    L.gcvo_eval_fgh_batch.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    L.gcvo_strerror.argtypes = [ctypes.c_int]
    L.gcvo_strerror.restype = ctypes.c_char_p
    L.gcvo_abi_version.argtypes = []
    L.gcvo_mlp_param_count.argtypes = []
    L.gcvo_mlp_param_count.restype = ctypes.c_longlong
    L.gcvo_mlp_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int]
    L.gcvo_mlp_workspace_size.restype = ctypes.c_size_t
    bp = ctypes.POINTER(gcvo_mlp_batch)
    L.gcvo_mlp_forward.argtypes = [bp, _P, _P, _P, _P, ctypes.c_size_t, _P]
    L.gcvo_mlp_loss_grad.argtypes = [bp, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    L.gcvo_mlp_adam.argtypes = [_P, _P, _P, _P, _P, ctypes.c_longlong, ctypes.c_int, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]
    _lib = L
    return L


def strerror(status: int) -> str:
    return load_library().gcvo_strerror(int(status)).decode()


def default_params(**overrides) -> gcvo_params:
    p = gcvo_params()
    load_library().gcvo_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_from_spec(spec, **overrides) -> gcvo_params:
    """gcvo_params from a ``synth.PairSpec``'s solver settings."""
    d = spec.params()
    d.update(overrides)
    return default_params(**d)


# ----------------------------------------------------------------- device plumbing

def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _cloud(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch CUDA tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3:
        raise TypeError(f"{name} must be float32 [n, 3]")
    return t.contiguous()


def _shape6(t, n: int, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != (6, n):
        raise TypeError(f"{name} must be a float32 CUDA tensor [6, {n}]")
    return t.contiguous()


def _labels(t, n: int, name: str):
    """Label rows: float32 CUDA [n, d], 1 <= d <= GCVO_MAX_LABEL_DIM."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 \
            or t.shape[0] != n or not 1 <= t.shape[1] <= GCVO_MAX_LABEL_DIM:
        raise TypeError(f"{name} must be a float32 CUDA tensor [{n}, d], 1 <= d <= {GCVO_MAX_LABEL_DIM}")
    return t.contiguous()


def workspace(nbytes: int, device=None):
    """A device byte buffer from torch's allocator (256-byte aligned)."""
    torch = _torch()
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, int(nbytes)


def _pose(T) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(4, 4))
    return a


# ----------------------------------------------------------------- entry points

def gcvo_workspace_size(n_tgt: int, n_src: int, params: gcvo_params) -> int:
    return int(load_library().gcvo_workspace_size(n_tgt, n_src, ctypes.byref(params)))


def gcvo_register(target, source, T_init=None, params: gcvo_params | None = None, ws=None, stream=None):
    """Register one pair; returns (T float64 4x4, info dict).  Raises GcvoError."""
    L = load_library()
    target = _cloud(target, "target")
    source = _cloud(source, "source")
    p = params if params is not None else default_params()
    T0 = None if T_init is None else _pose(T_init)
    need = L.gcvo_workspace_size(target.shape[0], source.shape[0], ctypes.byref(p))
    if ws is None:
        holder, wptr, wbytes = workspace(max(need, 256), target.device)
    else:
        holder, wptr, wbytes = ws
    T_out = np.zeros((4, 4))
    info = gcvo_info()
    st = L.gcvo_register(_ptr(target), target.shape[0], _ptr(source), source.shape[0],
                         T0.ctypes.data_as(_P) if T0 is not None else None, ctypes.byref(p),
                         T_out.ctypes.data_as(_P), ctypes.byref(info), ctypes.c_void_p(wptr), wbytes,
                         _stream_handle(stream))
    del holder
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_register")
    return T_out, info.to_dict()


def gcvo_batch_workspace_size(tgt_off, src_off, params) -> int:
    L = load_library()
    to = np.ascontiguousarray(tgt_off, dtype=np.int64)
    so = np.ascontiguousarray(src_off, dtype=np.int64)
    shared, parr = _param_array(params, len(to) - 1)
    return int(L.gcvo_batch_workspace_size(len(to) - 1, to.ctypes.data_as(_P), so.ctypes.data_as(_P), parr, shared))


def _param_array(params, n_pairs):
    if isinstance(params, gcvo_params):
        return 1, ctypes.pointer(params)
    arr = (gcvo_params * n_pairs)(*params)
    return 0, ctypes.cast(arr, ctypes.POINTER(gcvo_params))


def _device_poses(T, n_pairs: int, device):
    """Start poses as a float64 CUDA tensor [n_pairs, 16] (None stays None):
    a CUDA tensor is used in place, host values are copied over."""
    if T is None:
        return None
    torch = _torch()
    if isinstance(T, torch.Tensor) and T.is_cuda:
        if T.dtype != torch.float64 or T.numel() != 16 * n_pairs:
            raise TypeError(f"T_init must be float64 with {n_pairs} x 16 entries")
        return T.reshape(n_pairs, 16).contiguous()
    a = np.ascontiguousarray(np.asarray(T, np.float64).reshape(n_pairs, 16))
    return torch.from_numpy(a).to(device)


INFO_BYTES = ctypes.sizeof(gcvo_info)


def infos_from_device(buf) -> list:
    """Info dicts from a device gcvo_info array (uint8 CUDA tensor [n, INFO_BYTES])."""
    raw = buf.cpu().numpy().tobytes()
    return [gcvo_info.from_buffer_copy(raw, k * INFO_BYTES).to_dict() for k in range(len(raw) // INFO_BYTES)]


def _register_batch(targets, tgt_labels, tgt_off, sources, src_labels, src_off, T_init, params, ws, stream,
                    device):
    L = load_library()
    torch = _torch()
    targets = _cloud(targets, "targets")
    sources = _cloud(sources, "sources")
    to = np.ascontiguousarray(tgt_off, dtype=np.int64)
    so = np.ascontiguousarray(src_off, dtype=np.int64)
    n_pairs = len(to) - 1
    p = params if params is not None else default_params()
    shared, parr = _param_array(p, n_pairs)
    T0 = _device_poses(T_init, n_pairs, targets.device)
    T_out = torch.empty((n_pairs, 4, 4), dtype=torch.float64, device=targets.device)
    infos = torch.empty((n_pairs, INFO_BYTES), dtype=torch.uint8, device=targets.device)
    if tgt_labels is None:
        name = "gcvo_register_batch"
        need = L.gcvo_batch_workspace_size(n_pairs, to.ctypes.data_as(_P), so.ctypes.data_as(_P), parr, shared)
    else:
        name = "gcvo_register_batch_labeled"
        tl = _labels(tgt_labels, targets.shape[0], "tgt_labels")
        sl = _labels(src_labels, sources.shape[0], "src_labels")
        if tl.shape[1] != sl.shape[1]:
            raise TypeError("tgt_labels and src_labels must have the same width")
        dim = int(tl.shape[1])
        need = L.gcvo_batch_workspace_size_labeled(n_pairs, to.ctypes.data_as(_P), so.ctypes.data_as(_P), parr,
                                                   shared, dim)
    if ws is None:
        holder, wptr, wbytes = workspace(max(need, 256), targets.device)
    else:
        holder, wptr, wbytes = ws
    if tgt_labels is None:
        st = L.gcvo_register_batch(n_pairs, _ptr(targets), to.ctypes.data_as(_P), _ptr(sources),
                                   so.ctypes.data_as(_P), _ptr(T0), parr, shared, _ptr(T_out), _ptr(infos),
                                   ctypes.c_void_p(wptr), wbytes, _stream_handle(stream))
    else:
        st = L.gcvo_register_batch_labeled(n_pairs, _ptr(targets), _ptr(tl), to.ctypes.data_as(_P), _ptr(sources),
                                           _ptr(sl), so.ctypes.data_as(_P), dim, _ptr(T0), parr, shared,
                                           _ptr(T_out), _ptr(infos), ctypes.c_void_p(wptr), wbytes,
                                           _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, name)
    # the outputs are written on the stream after the call returns: keep the
    # workspace and the start poses alive until the stream has reached them
    s = torch.cuda.current_stream() if stream is None else stream
    if holder is not None:
        holder.record_stream(s)
    if T0 is not None:
        T0.record_stream(s)
    del holder
    if device:
        return T_out, infos
    return T_out.cpu().numpy(), infos_from_device(infos)


def gcvo_register_batch(targets, tgt_off, sources, src_off, T_init=None, params=None, ws=None, stream=None,
                        device: bool = False):
    """Register len(tgt_off) - 1 pairs held in two concatenated clouds.

    targets / sources: float32 CUDA [sum, 3]; tgt_off / src_off: int64 host
    offsets; T_init: None (identity), a float64 CUDA tensor [n_pairs, 4, 4]
    (used in place) or host values (copied to the device).  Returns (T, infos):
    with device=True a float64 CUDA tensor [n_pairs, 4, 4] and a uint8 CUDA
    tensor of gcvo_info records (see infos_from_device), both written on the
    stream; otherwise numpy [n_pairs, 4, 4] and a list of info dicts.
    """
    return _register_batch(targets, None, tgt_off, sources, None, src_off, T_init, params, ws, stream, device)


def gcvo_register_batch_labeled(targets, tgt_labels, tgt_off, sources, src_labels, src_off, T_init=None,
                                params=None, ws=None, stream=None, device: bool = False):
    """gcvo_register_batch with per-point label vectors (float32 CUDA [sum, d],
    d <= 4) weighting each pair by <l^X_i, l^Z_j>."""
    return _register_batch(targets, tgt_labels, tgt_off, sources, src_labels, src_off, T_init, params, ws, stream,
                           device)


def gcvo_batch_workspace_size_labeled(tgt_off, src_off, params, label_dim: int) -> int:
    L = load_library()
    to = np.ascontiguousarray(tgt_off, dtype=np.int64)
    so = np.ascontiguousarray(src_off, dtype=np.int64)
    shared, parr = _param_array(params, len(to) - 1)
    return int(L.gcvo_batch_workspace_size_labeled(len(to) - 1, to.ctypes.data_as(_P), so.ctypes.data_as(_P), parr,
                                                   shared, int(label_dim)))


@dataclass
class EvalResult:
    f: float
    g: np.ndarray
    H: np.ndarray
    npairs: int


def _eval_fgh(target, tgt_shape6, tgt_labels, source, src_shape6, src_labels, T, length_scale, cutoff, sigma2,
              precision, ws, stream) -> EvalResult:
    L = load_library()
    target = _cloud(target, "target")
    source = _cloud(source, "source")
    nt, ns = target.shape[0], source.shape[0]
    ts = _shape6(tgt_shape6, nt, "tgt_shape6")
    ss = _shape6(src_shape6, ns, "src_shape6")
    Tm = _pose(T)
    if tgt_labels is None:
        dim = 0
        need = L.gcvo_eval_workspace_size(nt, ns)
    else:
        tl = _labels(tgt_labels, nt, "tgt_labels")
        sl = _labels(src_labels, ns, "src_labels")
        if tl.shape[1] != sl.shape[1]:
            raise TypeError("tgt_labels and src_labels must have the same width")
        dim = int(tl.shape[1])
        need = L.gcvo_eval_workspace_size_labeled(nt, ns, dim)
    if ws is None:
        holder, wptr, wbytes = workspace(max(need, 256), target.device)
    else:
        holder, wptr, wbytes = ws
    f = ctypes.c_double()
    g = np.zeros(6)
    H = np.zeros((6, 6))
    npairs = ctypes.c_longlong()
    tail = (Tm.ctypes.data_as(_P), float(length_scale), float(cutoff), float(sigma2), int(precision), ctypes.byref(f),
            g.ctypes.data_as(_P), H.ctypes.data_as(_P), ctypes.byref(npairs), ctypes.c_void_p(wptr), wbytes,
            _stream_handle(stream))
    if dim == 0:
        name = "gcvo_eval_fgh"
        st = L.gcvo_eval_fgh(_ptr(target), _ptr(ts), nt, _ptr(source), _ptr(ss), ns, *tail)
    else:
        name = "gcvo_eval_fgh_labeled"
        st = L.gcvo_eval_fgh_labeled(_ptr(target), _ptr(ts), _ptr(tl), nt, _ptr(source), _ptr(ss), _ptr(sl), ns, dim,
                                     *tail)
    del holder
    if st != GCVO_OK:
        raise GcvoError(st, name)
    return EvalResult(f.value, g, H, npairs.value)


def gcvo_eval_fgh(target, tgt_shape6, source, src_shape6, T, length_scale: float, cutoff: float,
                  sigma2: float = 1.0, precision: int = GCVO_PRECISION_FP32, ws=None, stream=None) -> EvalResult:
    return _eval_fgh(target, tgt_shape6, None, source, src_shape6, None, T, length_scale, cutoff, sigma2, precision,
                     ws, stream)


def gcvo_eval_fgh_noalloc(target, tgt_shape6, source, src_shape6, T, length_scale: float, cutoff: float,
                          sigma2: float = 1.0, precision: int = GCVO_PRECISION_FP32, stream=None) -> EvalResult:
    """gcvo_eval_fgh with the library's per-GPU scratch instead of a workspace
    (no device allocation; sizes beyond GCVO_NOALLOC_SCRATCH_BYTES raise
    GCVO_ERR_CAPACITY; overlapping calls on one GPU race)."""
    L = load_library()
    target = _cloud(target, "target")
    source = _cloud(source, "source")
    nt, ns = target.shape[0], source.shape[0]
    ts = _shape6(tgt_shape6, nt, "tgt_shape6")
    ss = _shape6(src_shape6, ns, "src_shape6")
    Tm = _pose(T)
    f = ctypes.c_double()
    g = np.zeros(6)
    H = np.zeros((6, 6))
    npairs = ctypes.c_longlong()
    st = L.gcvo_eval_fgh_noalloc(_ptr(target), _ptr(ts), nt, _ptr(source), _ptr(ss), ns, Tm.ctypes.data_as(_P),
                                 float(length_scale), float(cutoff), float(sigma2), int(precision), ctypes.byref(f),
                                 g.ctypes.data_as(_P), H.ctypes.data_as(_P), ctypes.byref(npairs),
                                 _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_eval_fgh_noalloc")
    return EvalResult(f.value, g, H, npairs.value)


def gcvo_eval_fgh_labeled(target, tgt_shape6, tgt_labels, source, src_shape6, src_labels, T, length_scale: float,
                          cutoff: float, sigma2: float = 1.0, precision: int = GCVO_PRECISION_FP32, ws=None,
                          stream=None) -> EvalResult:
    """gcvo_eval_fgh with per-point label vectors weighting each pair."""
    return _eval_fgh(target, tgt_shape6, tgt_labels, source, src_shape6, src_labels, T, length_scale, cutoff, sigma2,
                     precision, ws, stream)


def gcvo_eval_workspace_size_labeled(n_tgt: int, n_src: int, label_dim: int) -> int:
    return int(load_library().gcvo_eval_workspace_size_labeled(n_tgt, n_src, label_dim))


def gcvo_point_shapes(xyz, knn: int = 10, rho: float = 0.01, ws=None, stream=None):
    """Per-point shapes, float32 CUDA [6, n] (enqueued on the stream)."""
    torch = _torch()
    L = load_library()
    xyz = _cloud(xyz, "xyz")
    n = xyz.shape[0]
    out = torch.empty((6, n), dtype=torch.float32, device=xyz.device)
    need = L.gcvo_shapes_workspace_size(n)
    if ws is None:
        holder, wptr, wbytes = workspace(max(need, 256), xyz.device)
    else:
        holder, wptr, wbytes = ws
    st = L.gcvo_point_shapes(_ptr(xyz), n, int(knn), float(rho), _ptr(out), ctypes.c_void_p(wptr), wbytes,
                             _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_point_shapes")
    # keep the workspace alive until the kernels have run
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    del holder
    return out


def gcvo_point_shapes_batch(xyz, off, knn: int = 10, rho: float = 0.01, stream=None):
    """Shapes of the clouds xyz[off[k]:off[k+1]] (float32 CUDA [sum, 3], host
    offsets): float32 CUDA [6 * sum], cloud k's [6, n_k] block at 6 * off[k]."""
    torch = _torch()
    L = load_library()
    xyz = _cloud(xyz, "xyz")
    o = np.ascontiguousarray(off, dtype=np.int64)
    out = torch.empty(6 * xyz.shape[0], dtype=torch.float32, device=xyz.device)
    need = L.gcvo_shapes_batch_workspace_size(len(o) - 1, o.ctypes.data_as(_P))
    holder, wptr, wbytes = workspace(max(need, 256), xyz.device)
    st = L.gcvo_point_shapes_batch(len(o) - 1, _ptr(xyz), o.ctypes.data_as(_P), int(knn), float(rho), _ptr(out),
                                   ctypes.c_void_p(wptr), wbytes, _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_point_shapes_batch")
    holder.record_stream(torch.cuda.current_stream() if stream is None else stream)
    return out


def shape_block(shapes, off, k: int):
    """Cloud k's [6, n_k] view of a gcvo_point_shapes_batch output."""
    a, b = int(off[k]), int(off[k + 1])
    return shapes[6 * a:6 * b].view(6, b - a)


@dataclass
class EvalBatch:
    f: object        # float64 CUDA [n]
    g: object        # float64 CUDA [n, 6]
    H: object        # float64 CUDA [n, 6, 6]
    npairs: object   # int64 CUDA [n]
    status: object   # int32 CUDA [n]


def gcvo_eval_fgh_batch(targets, tgt_shapes, tgt_off, sources, src_shapes, src_off, T, length_scales,
                        cutoff_scale: float = 3.0, sigma2: float = 1.0, precision: int = GCVO_PRECISION_FP32,
                        stream=None) -> EvalBatch:
    """Evaluations of several pairs in one pass: shapes in the layout of
    gcvo_point_shapes_batch, T None (identity) or float64 CUDA [n, 4, 4] (or
    host values, copied over), length_scales host [n].  Outputs stay on the
    device."""
    torch = _torch()
    L = load_library()
    targets = _cloud(targets, "targets")
    sources = _cloud(sources, "sources")
    to = np.ascontiguousarray(tgt_off, dtype=np.int64)
    so = np.ascontiguousarray(src_off, dtype=np.int64)
    n = len(to) - 1
    for name, sh, rows in (("tgt_shapes", tgt_shapes, targets.shape[0]), ("src_shapes", src_shapes, sources.shape[0])):
        if not sh.is_cuda or sh.dtype != torch.float32 or sh.numel() != 6 * rows:
            raise TypeError(f"{name} must be a float32 CUDA tensor of 6 x {rows} values")
    ells = np.ascontiguousarray(np.broadcast_to(np.asarray(length_scales, np.float64), (n,)))
    T0 = _device_poses(T, n, targets.device)
    dev = targets.device
    out = EvalBatch(torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, 6), dtype=torch.float64, device=dev),
                    torch.empty((n, 6, 6), dtype=torch.float64, device=dev),
                    torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    need = L.gcvo_eval_batch_workspace_size(n, to.ctypes.data_as(_P), so.ctypes.data_as(_P))
    holder, wptr, wbytes = workspace(max(need, 256), dev)
    st = L.gcvo_eval_fgh_batch(n, _ptr(targets), _ptr(tgt_shapes.contiguous()), to.ctypes.data_as(_P), _ptr(sources),
                               _ptr(src_shapes.contiguous()), so.ctypes.data_as(_P), _ptr(T0),
                               ells.ctypes.data_as(_P), float(cutoff_scale), float(sigma2), int(precision),
                               _ptr(out.f), _ptr(out.g), _ptr(out.H), _ptr(out.npairs), _ptr(out.status),
                               ctypes.c_void_p(wptr), wbytes, _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_eval_fgh_batch")
    s = torch.cuda.current_stream() if stream is None else stream
    holder.record_stream(s)
    if T0 is not None:
        T0.record_stream(s)
    return out


def profiled(params, profile: gcvo_profile):
    """Copy of a parameter set (or list of them) whose calls add their
    pair-kernel measurement to ``profile``."""
    def one(p):
        q = gcvo_params()
        ctypes.pointer(q)[0] = p
        q.profile = ctypes.pointer(profile)
        return q
    return one(params) if isinstance(params, gcvo_params) else [one(p) for p in params]


# ------------------------------------------------------------ warm-start network

class MlpBatch:
    """Inputs of one network call: two device clouds with the host row ranges
    (start, count) of every sample's target and source, device int32 row
    indices [B, P] within those ranges, optional device float32 target and
    source motions [B, 12], and the input scale in metres.  Holds references to every array it
    points at."""

    def __init__(self, targets, tgt_start, tgt_count, sources, src_start, src_count, tgt_idx, src_idx,
                 tgt_motion=None, src_motion=None, input_scale: float = 20.0):
        torch = _torch()
        self.targets = _cloud(targets, "targets")
        self.sources = _cloud(sources, "sources")
        self.ranges = [np.ascontiguousarray(a, dtype=np.int64) for a in (tgt_start, tgt_count, src_start, src_count)]
        B = len(self.ranges[0])
        if any(len(r) != B for r in self.ranges):
            raise TypeError("row ranges must all have one entry per sample")
        for name, t in (("tgt_idx", tgt_idx), ("src_idx", src_idx)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 or t.dim() != 2 \
                    or t.shape[0] != B:
                raise TypeError(f"{name} must be an int32 CUDA tensor [{B}, P]")
        self.tgt_idx = tgt_idx.contiguous()
        self.src_idx = src_idx.contiguous()
        if self.tgt_idx.shape != self.src_idx.shape:
            raise TypeError("tgt_idx and src_idx must have the same shape")
        self.motions = []
        for name, m in (("tgt_motion", tgt_motion), ("src_motion", src_motion)):
            if m is not None and (not m.is_cuda or m.dtype != torch.float32 or tuple(m.shape) != (B, 12)):
                raise TypeError(f"{name} must be a float32 CUDA tensor [{B}, 12]")
            self.motions.append(m.contiguous() if m is not None else None)
        r = self.ranges
        self.c = gcvo_mlp_batch(B, int(self.tgt_idx.shape[1]), self.targets.data_ptr(), self.targets.shape[0],
                                r[0].ctypes.data, r[1].ctypes.data, self.sources.data_ptr(), self.sources.shape[0],
                                r[2].ctypes.data, r[3].ctypes.data, self.tgt_idx.data_ptr(), self.src_idx.data_ptr(),
                                *[m.data_ptr() if m is not None else None for m in self.motions],
                                float(input_scale))

    @property
    def n_pairs(self) -> int:
        return self.c.n_pairs


def gcvo_mlp_workspace_size(n_pairs: int, n_points: int) -> int:
    return int(load_library().gcvo_mlp_workspace_size(int(n_pairs), int(n_points)))


def gcvo_mlp_forward(batch: MlpBatch, w_bf16, poses: bool = False, ws=None, stream=None):
    """Network outputs (float32 CUDA [B, 6]) and, with poses=True, the predicted
    poses exp(xi^) as a float64 CUDA tensor [B, 4, 4]."""
    torch = _torch()
    L = load_library()
    B, P = batch.c.n_pairs, batch.c.n_points
    out = torch.empty((B, 6), dtype=torch.float32, device=batch.targets.device)
    holder, wptr, wbytes = ws if ws is not None else workspace(max(gcvo_mlp_workspace_size(B, P), 256),
                                                              batch.targets.device)
    T = torch.empty((B, 4, 4), dtype=torch.float64, device=batch.targets.device) if poses else None
    st = L.gcvo_mlp_forward(ctypes.byref(batch.c), _ptr(w_bf16), _ptr(out), _ptr(T), ctypes.c_void_p(wptr), wbytes,
                            _stream_handle(stream))
    del holder
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_mlp_forward")
    return (out, T) if poses else out


def gcvo_mlp_loss_grad(batch: MlpBatch, w_bf16, y6, grad=None, loss=None, out6=None, ws=None, stream=None):
    """Loss (float32 CUDA [1]) and gradient (float32 CUDA [n_params])."""
    torch = _torch()
    L = load_library()
    dev = batch.targets.device
    B, P = batch.c.n_pairs, batch.c.n_points
    if not y6.is_cuda or y6.dtype != torch.float32 or tuple(y6.shape) != (B, 6):
        raise TypeError(f"y6 must be a float32 CUDA tensor [{B}, 6]")
    y6 = y6.contiguous()
    grad = grad if grad is not None else torch.empty(GCVO_MLP_N_PARAMS, dtype=torch.float32, device=dev)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=dev)
    holder, wptr, wbytes = ws if ws is not None else workspace(max(gcvo_mlp_workspace_size(B, P), 256), dev)
    st = L.gcvo_mlp_loss_grad(ctypes.byref(batch.c), _ptr(w_bf16), _ptr(y6), _ptr(out6), _ptr(loss), _ptr(grad),
                              ctypes.c_void_p(wptr), wbytes, _stream_handle(stream))
    del holder
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_mlp_loss_grad")
    return loss, grad


def gcvo_mlp_adam(w, w_bf16, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None) -> None:
    L = load_library()
    st = L.gcvo_mlp_adam(_ptr(w), _ptr(w_bf16), _ptr(m), _ptr(v), _ptr(grad), int(w.numel()), int(step),
                         float(lr), float(beta1), float(beta2), float(eps), _stream_handle(stream))
    if st != GCVO_OK:
        raise GcvoError(st, "gcvo_mlp_adam")
