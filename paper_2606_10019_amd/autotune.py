"""Cell-size autotuner for the pair kernel.

The pair grid's cell edge (``gcvo_params.cell_fraction``, a fraction of the
cutoff radius) trades the candidates a source point walks (large cells: more
targets outside the cutoff) against the cell rows it lists (small cells: more,
shorter rows).  Every value finds the same pairs within the cutoff, so the
choice changes speed, not the sums beyond the order of FP32 additions.  The
tuner times whole registrations (one batch call over sample pairs) for each
candidate fraction on the device and returns the fastest; the caller then
passes it in its parameters, so results stay reproducible call to call.
"""
from __future__ import annotations

import ctypes
import time

from . import gcvo

CANDIDATES = (0.25, 0.35, 0.5, 0.7, 1.0)


def _with_fraction(params, frac: float):
    def one(p):
        q = gcvo.gcvo_params()
        ctypes.pointer(q)[0] = p
        q.cell_fraction = frac
        return q
    if isinstance(params, gcvo.gcvo_params):
        return one(params)
    return [one(p) for p in params]


def autotune_cell_fraction(targets, tgt_off, sources, src_off, params, candidates=CANDIDATES, reps: int = 3,
                           T_init=None):
    """Time gcvo_register_batch over the given pairs for every candidate cell
    fraction.  Returns (best fraction, {fraction: milliseconds per call},
    {fraction: list of info dicts of the last call})."""
    import torch
    timings, infos = {}, {}
    for frac in candidates:
        p = _with_fraction(params, frac)
        ws = gcvo.workspace(gcvo.gcvo_batch_workspace_size(tgt_off, src_off, p), targets.device)
        gcvo.gcvo_register_batch(targets, tgt_off, sources, src_off, T_init, p, ws=ws)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, info = gcvo.gcvo_register_batch(targets, tgt_off, sources, src_off, T_init, p, ws=ws)
        torch.cuda.synchronize()
        timings[frac] = 1e3 * (time.perf_counter() - t0) / reps
        infos[frac] = info
    best = min(timings, key=timings.get)
    return best, timings, infos
