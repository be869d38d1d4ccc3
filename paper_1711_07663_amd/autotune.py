"""Autotuner of the batched cut's launch parameters.

Two knobs change speed, never results (every setting gives the same
iblank): the cap on a surface's bins per axis (coarser bins hold more faces
each, so bin walks get longer but bin arrays smaller) and the number of
wavefronts the persistent exact-stage kernels launch.  The tuner groups the
cuts of a batch into size classes by face count (octaves), times each class
alone under each bin-cap factor and keeps the fastest, then times the whole
batch under each wavefront count.  Results can be saved and reloaded as
JSON keyed by size class.
"""
from __future__ import annotations

import json
import math
import time

import torch

from . import oc as _oc


def size_class(n_face):
    """Octave of the face count (384 -> 9, 24 576 -> 15)."""
    return int(math.floor(math.log2(max(int(n_face), 1))))


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def apply(ctx, surf_faces, params):
    """Apply tuned parameters: surf_faces maps surface id -> face count."""
    auto = {}
    for sid in surf_faces:
        auto[sid] = ctx.tune(_oc.OC_TUNE_SURF_BINS, sid, 0)
    for sid, nf in surf_faces.items():
        f = params.get("bin_factor", {}).get(str(size_class(nf)), 1.0)
        ctx.tune(_oc.OC_TUNE_SURF_BINS, sid, max(1, int(round(auto[sid] * f))))
    ctx.tune(_oc.OC_TUNE_EXACT_WAVES, 0, int(params.get("exact_waves", 0)))


def tune_batch(ctx, reqs, surf_faces, factors=(1.0, 0.75, 0.5), waves=(2048, 4096, 8192, 16384), reps=3):
    """reqs: [(grid_id, [surf_id], host poses [1,12], iblank)] cut with
    Context.cut_batch (default slot).  Returns the chosen parameters and
    the timings behind them."""
    auto = {sid: ctx.tune(_oc.OC_TUNE_SURF_BINS, sid, 0) for sid in surf_faces}
    classes = {}
    for r in reqs:
        for sid in r[1]:
            classes.setdefault(size_class(surf_faces[sid]), []).append(r)
    report = dict(classes={}, waves={})
    chosen = {}
    for c, sub in sorted(classes.items()):
        sids = sorted({sid for r in sub for sid in r[1]})
        times = {}
        for f in factors:
            for sid in sids:
                ctx.tune(_oc.OC_TUNE_SURF_BINS, sid, max(1, int(round(auto[sid] * f))))
            times[f] = _time(lambda: ctx.cut_batch(sub), reps)
        best = min(times, key=times.get)
        chosen[str(c)] = best
        for sid in sids:
            ctx.tune(_oc.OC_TUNE_SURF_BINS, sid, max(1, int(round(auto[sid] * best))))
        report["classes"][str(c)] = dict(cuts=len(sub), ms={str(k): 1e3 * v for k, v in times.items()}, factor=best)
    wt = {}
    for w in waves:
        ctx.tune(_oc.OC_TUNE_EXACT_WAVES, 0, w)
        wt[w] = _time(lambda: ctx.cut_batch(reqs), reps)
    best_w = min(wt, key=wt.get)
    ctx.tune(_oc.OC_TUNE_EXACT_WAVES, 0, best_w)
    report["waves"] = {str(k): 1e3 * v for k, v in wt.items()}
    params = dict(bin_factor=chosen, exact_waves=best_w)
    return params, report


def save(params, path):
    with open(path, "w") as f:
        json.dump(params, f, indent=1, sort_keys=True)


def load(path):
    with open(path) as f:
        return json.load(f)
