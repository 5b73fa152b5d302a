"""Cell-shape autotuner for the pair kernel.

The pair grid's cells have an edge along y and z (``gcvo_params.cell_fraction``)
and along x, the direction of the rows a source point walks
(``cell_fraction_x``), both as fractions of the cutoff radius.  Larger cells
make a point walk more targets outside its cutoff; smaller y-z cells add rows
to list and switch between; smaller x cells clip each row closer to the cutoff
ball at no extra rows but with more cells.  Every shape finds the same pairs
within the cutoff, so the choice changes speed, not the sums beyond the order
of FP32 additions.  The tuner times whole registrations (one batch call over
sample pairs) for each candidate shape on the device and returns the fastest;
the caller then passes it in its parameters, so results stay reproducible
call to call.
"""
from __future__ import annotations

import ctypes
import time

from . import gcvo

# (y-z fraction, x fraction)
CANDIDATES = ((0.35, 0.35), (0.35, 0.125), (0.5, 0.5), (0.5, 0.25), (0.5, 0.125), (0.7, 0.7), (0.7, 0.25),
              (0.7, 0.125), (1.0, 0.25))


def _with_fraction(params, frac):
    fyz, fx = (frac, frac) if isinstance(frac, (int, float)) else frac

    def one(p):
        q = gcvo.gcvo_params()
        ctypes.pointer(q)[0] = p
        q.cell_fraction = fyz
        q.cell_fraction_x = fx
        return q
    if isinstance(params, gcvo.gcvo_params):
        return one(params)
    return [one(p) for p in params]


def autotune_cell_fraction(targets, tgt_off, sources, src_off, params, candidates=CANDIDATES, reps: int = 3,
                           T_init=None):
    """Time gcvo_register_batch over the given pairs for every candidate cell
    shape (a (y-z, x) pair of fractions, or one fraction for cubic cells).
    Returns (best candidate, {candidate: milliseconds per call},
    {candidate: list of info dicts of the last call})."""
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
