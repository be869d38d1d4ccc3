"""Autotuner of the batched cut's launch parameters.

Three knobs change speed, never results (every setting gives the same
iblank): the cap on a surface's bins per axis (coarser bins hold more faces
each, so bin walks get longer but bin arrays smaller), the number of
wavefronts the persistent exact-stage kernels launch, and the block shape
of the streaming element filter (threads per block, four elements each).
The tuner groups the cuts of a batch into size classes by face count
(octaves), times each class alone under each bin-cap factor and keeps the
fastest, then times the whole batch under each wavefront count and each
filter block.  ``save`` writes the tuning file a context reads at creation
(``Context(tune_cache=path)``, oc_config.tune_cache): one "key value" line
per knob, "bin_factor <octave> <factor>" per size class.
"""
from __future__ import annotations

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
    ctx.tune(_oc.OC_TUNE_FILTER_BLOCK, 0, int(params.get("filter_block", 0)))


def tune_batch(ctx, reqs, surf_faces, factors=(1.0, 0.75, 0.5), waves=(2048, 4096, 8192, 16384),
               blocks=(128, 256, 512, 1024), reps=3):
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
    bt = {}
    for b in blocks:
        ctx.tune(_oc.OC_TUNE_FILTER_BLOCK, 0, b)
        bt[b] = _time(lambda: ctx.cut_batch(reqs), reps)
    best_b = min(bt, key=bt.get)
    ctx.tune(_oc.OC_TUNE_FILTER_BLOCK, 0, best_b)
    report["filter_block"] = {str(k): 1e3 * v for k, v in bt.items()}
    params = dict(bin_factor=chosen, exact_waves=best_w, filter_block=best_b)
    return params, report


def save(params, path):
    """Write params as the library's tuning file (oc_config.tune_cache)."""
    lines = ["# overset cut tuning: knob value (bin_factor: face-count octave, factor)"]
    for k in ("exact_waves", "filter_block", "donor_waves"):
        if k in params:
            lines.append("%s %d" % (k, int(params[k])))
    for c, f in sorted(params.get("bin_factor", {}).items(), key=lambda kv: int(kv[0])):
        lines.append("bin_factor %d %.17g" % (int(c), float(f)))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def load(path):
    """Read a tuning file back into params."""
    params = dict(bin_factor={})
    with open(path) as f:
        for line in f:
            t = line.split("#", 1)[0].split()
            if not t:
                continue
            if t[0] == "bin_factor":
                params["bin_factor"][str(int(t[1]))] = float(t[2])
            else:
                params[t[0]] = int(t[1])
    return params
