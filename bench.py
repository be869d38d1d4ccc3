"""Benchmark: the overset connectivity hot path on one MI355X.

Default workload (the single dimpled-sphere cut): background 128^3 quadratic
hexes on [-3,3]^3 with the sinusoidal displacement; cut surface: R = 0.5
sphere with 300 spherical-cap dimples, 24 576 quadratic quads; near-body shell
of 8 layers (196 608 hexes) to r = 1.  A step is the whole hot path: pose,
bins, filter, exact intersection, nearest-face side, ray parity, union, fringe
marking, Gauss receptor points and Newton donor search in both directions.
Inputs are generated from fixed formulas (synthetic), resident on the device
before timing.

Other workloads (--workload):
  spin   the dimpled sphere spinning about z at one turn per 400 steps, 200
         steps, each a warm-started re-cut plus donors, replayed as HIP graphs;
  batch  64 uneven instances (SeedSequence(1711)) cut in one launch per stage,
         against the same instances cut one at a time;
  serve  Poisson arrivals over four device-resident grid sets served with
         continuous batching, against one-at-a-time service;
  ab     the dimpled case with the receptors of the artificial-boundary
         method: AB faces of the background and of the shell, 3 x 3 Gauss
         flux points per face, their donors and 27 interpolation weights per
         point, both directions, replayed as a HIP graph;
  filtered  the paper's own filtered cut of the dimpled 128^3 case (N_F^1,
         N_F^2 = 16,4 / 4,1 / 1,1) against the exact cut: time per cut
         and the elements on which the truncations change the blanking;
  refined  the cut with the curved faces resolved to level k (faces split
         k x k, near elements k^3 times) of the dimpled 128^3 case against
         the lattice cut: time per cut and the elements whose blanking the
         curvature changes;
  unblank  the dimpled sphere turning and oscillating (amplitude 0.5) through
         the background: per step the background is cut at the poses of t
         and t + dt (wall rule: union of holes), the cells to unblank are
         listed, and their 27 interior points get donors in the shell.

Prints one JSON line.  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_VECTOR_PEAK = 78.6        # TFLOP/s, MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
# algorithmic FLOP per Newton iteration of the donor search: the per-unit
# figure of the method's Newton step, x(xi) and J = dx/dxi of a 27-node
# element (27 nodes x 4 values x 3 components multiply-adds) plus the 3x3
# solve, about 0.7 kFLOP; the kernel evaluates the same map from its
# monomial coefficients by nested Horner steps (49 multiply-adds per
# coordinate)
NEWTON_FLOP = 700


KERNEL_SOURCE = {"k_dp_newton": "paper_1711_07663_amd/csrc/k_donor.hip", "k_dp_count": "paper_1711_07663_amd/csrc/k_donor.hip",
                 "k_filter": "paper_1711_07663_amd/csrc/k_cut.hip"}
# headers every kernel source includes (their device functions are part of the kernels)
KERNEL_HEADERS = ["paper_1711_07663_amd/csrc/dev_common.h", "paper_1711_07663_amd/csrc/dev_geom.h",
                  "paper_1711_07663_amd/csrc/q2.h", "paper_1711_07663_amd/csrc/oc_internal.h", "include/oc.h"]


def _code_only(text):
    """C/C++ source with its comments removed and its whitespace collapsed, so
    that an edit of a comment does not count as a change of the code."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha(kernel):
    """SHA-256 of the code ``kernel`` is compiled from, comments aside: its
    source file and the shared headers (so a change to a device function it
    calls counts)."""
    import hashlib
    src = KERNEL_SOURCE.get(kernel)
    if not src:
        return None
    h = hashlib.sha256()
    for f in [src] + KERNEL_HEADERS:
        path = f if os.path.isabs(f) else os.path.join(ROOT, f)
        if not os.path.exists(path):
            return None
        h.update(_code_only(open(path, encoding="utf-8").read()).encode())
    return h.hexdigest()


def filter_bytes(grid, surf_nodes, pose, wave=256):
    """Bytes k_filter moves for the cut of ``grid`` by a surface at ``pose``
    (grid frame): every wavefront of 256 consecutive elements reads their
    union box (24 B); if it meets the surface box, the z planes of the
    elements' FP32 boxes (8 B per element), then the y planes only if some
    element's z range meets the surface box, the x planes only if some
    element meets it in z and y; every element's iblank byte is written, and
    a ragged tail reads the planes of its elements.  The boxes are the node
    boxes and the surface box is the posed nodes' box widened by 1e-5 (the
    kernel's FP32 boxes round outward by less), so this models the kernel's
    early exits on the host."""
    R = np.asarray(pose[:9], dtype=np.float64).reshape(3, 3)
    Y = np.asarray(surf_nodes, dtype=np.float64) @ R.T + np.asarray(pose[9:12], dtype=np.float64)
    slo, shi = Y.min(axis=0) - 1e-5, Y.max(axis=0) + 1e-5
    n = grid.n_elem
    nw = n // wave
    full = nw * wave
    lo, hi = [], []
    for d in range(3):
        c = grid.nodes[:, d][grid.conn[:full]]
        lo.append(c.min(axis=1))
        hi.append(c.max(axis=1))
        del c
    meets = np.ones(nw, dtype=bool)
    for d in range(3):
        meets &= (lo[d].reshape(nw, wave).min(axis=1) <= shi[d]) & (hi[d].reshape(nw, wave).max(axis=1) >= slo[d])
    live = np.repeat(meets, wave)
    nbytes = 24.0 * (nw + (n > full))
    for d in (2, 1, 0):
        nbytes += 8.0 * wave * int(live.reshape(nw, wave).any(axis=1).sum())
        live &= (lo[d] <= shi[d]) & (hi[d] >= slo[d])
    return nbytes + 24.0 * (n - full) + 1.0 * n


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed profiler
    summary profiles/<kernel>_traffic_dimpled128.md (FETCH_SIZE and
    WRITE_SIZE passes scaled by the copy-kernel calibration), or None when
    there is none or the kernel's definition changed since it was taken
    (the summary records the SHA-256 of the kernel's sources)."""
    path = os.path.join(ROOT, "profiles", "%s_traffic_dimpled128.md" % kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    try:
        if vals.get("kernel_source_sha256") != kernel_source_sha(kernel):
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError, OSError, StopIteration):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1, help="oracle runs on every k-th element / point")
    ap.add_argument("--bg", type=int, default=128)
    ap.add_argument("--workload", default="dimpled",
                    choices=["dimpled", "spin", "batch", "serve", "service", "unblank", "ab", "filtered", "refined"])
    ap.add_argument("--levels", default="1,2,4", help="refined: levels k of the curved-face cut")
    ap.add_argument("--spin-steps", type=int, default=200)
    ap.add_argument("--topology", default="walls", choices=["walls", "paper"],
                    help="ab: the background cut by the walls, or by the shells' overset boundaries")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--rates", default="50,100,200,500", help="serve: arrival rates, requests/s")
    ap.add_argument("--requests", type=int, default=2000, help="serve, service: requests per rate")
    ap.add_argument("--service-rates", default="500,1000,2000,4000", help="service: arrival rates, requests/s")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="default workload: requests of the short serving segment (0: none)")
    ap.add_argument("--serve-rate", type=float, default=500.0, help="default workload: its arrival rate, req/s")
    ap.add_argument("--surf-bins", type=float, default=0.0,
                    help="scale of the wall's bins per axis (0: the library's choice)")
    ap.add_argument("--exact-waves", type=int, default=0,
                    help="wavefronts of the persistent exact-stage kernels (0: the library default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 512 MiB device-to-device copy (calibrates profiler byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(case, sample_every):
    """The oracle, as it stands, on the same step: cut of the background
    (every sample_every-th element; 1 = all), fringe layer, receptor points
    and donors of the background fringe in the shell, the shell's overset
    fringe, its receptor points and their donors in the background (every
    sample_every-th point).  The step time is scaled by sample_every."""
    import oracle as O
    bg = case["bg"]
    body = case["bodies"][0]
    s, sh = body["surface"], body["shell"]
    pose = case["poses"][0]
    O.build(force=False)
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        pass
    threads = min(threads, 16)
    k = max(1, int(sample_every))
    t0 = time.perf_counter()
    sel = np.arange(0, bg.n_elem, k, dtype=np.int64)
    st = O.cut_surface(bg, s, pose, sel=sel, threads=threads)
    hole = np.zeros(bg.n_elem, dtype=bool)
    hole[sel] = st == 0
    ib = O.mark_fringe(hole, O.face_neighbors(bg.conn))
    pts_bg = O.fringe_points(bg, O.fringe_elements(ib))
    d_bg, r_bg, _ = O.donor_search(sh, pts_bg[::k], pose, threads=threads)
    ib_sh = O.cut(sh, [], [])
    pts_sh = O.fringe_points(sh, O.fringe_elements(ib_sh), pose)
    d_sh, r_sh, _ = O.donor_search(bg, pts_sh[::k], threads=threads)
    t_wall = time.perf_counter() - t0
    t_step = t_wall * k
    what = "the whole step" if k == 1 else "every %d-th background element and receptor point (step time x %d)" % (k, k)
    return dict(value=bg.n_elem / t_step, unit="elements/s", cores=threads, kind="oracle",
                sample="%s: cut of the 128^3 background, fringe, %d + %d receptor points and their donors in "
                       "both directions; %.1f s of wall time on %d threads" % (what, pts_bg.shape[0],
                                                                              pts_sh.shape[0], t_wall, threads),
                t_step_s=t_step, results=dict(k=k, sel=sel, ib=ib, d_bg=d_bg, r_bg=r_bg, d_sh=d_sh, r_sh=r_sh))


def precision_report(snap, info, res):
    """How the FP32 stages and the FP64 path compare with the FP64 oracle on
    the same step: the share of the FP32 candidate filter's near elements that
    the exact test does not find intersected, and the iblank, donor ids and
    largest reference-coordinate difference against the oracle (when the
    oracle ran the whole step).  ``snap``: host copy of the outputs of the
    timed path (the last graph-replayed step)."""
    k = res["k"]
    ib_g = snap["ib_bg"]
    out = dict(filter_in_box=info["n_inbox"], filter_near=info["n_near"], exact_hit=info["n_hit"],
               near_not_hit_frac=(info["n_near"] - info["n_hit"]) / max(info["n_near"], 1))
    if k != 1:
        return out   # a sampled cut gives the oracle another fringe: nothing to compare point by point
    out["iblank_equal"] = bool(np.array_equal(ib_g, res["ib"]))
    b = snap["bodies"][0]
    err = 0.0
    same = True
    for d_o, r_o, dg, rg in ((res["d_bg"], res["r_bg"], b["donor_bg"], b["ref_bg"]),
                             (res["d_sh"], res["r_sh"], b["donor"], b["ref"])):
        n = d_o.shape[0]
        if dg.shape[0] != n:
            same = False
            continue
        d_g = dg[:n]
        r_g = rg[:n]
        same &= bool(np.array_equal(d_g, d_o))
        ok = (d_o >= 0) & (d_g == d_o)
        if ok.any():
            err = max(err, float(np.abs(r_g[ok] - r_o[ok]).max()))
    out["donor_ids_equal"] = same
    out["max_ref_coord_diff"] = err
    return out


def copy_ceiling_gbs(nbytes=1 << 29, reps=10):
    """HBM rate of a plain device-to-device copy (bytes read + written per
    second), the practical ceiling for a streaming kernel."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * nbytes / t / 1e9


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the method's multi-GPU sharding is a design note, "
              "not part of this build (got --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        import torch
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8))
        del src, dst
    out = dict(dimpled=run_dimpled, spin=run_spin, batch=run_batch, serve=run_serve, service=run_service,
               unblank=run_unblank, ab=run_ab, filtered=run_filtered, refined=run_refined)[a.workload](a)
    print(json.dumps(out), flush=True)


def run_dimpled(a):
    import torch
    from paper_1711_07663_amd import oc
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    from workloads import configs as CF

    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg = case["bg"]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    if a.exact_waves:
        ctx.tune(oc.OC_TUNE_EXACT_WAVES, 0, a.exact_waves)
    log("registering grids and surface")
    t0 = time.perf_counter()
    system = OversetSystem(ctx, case, bg_points_cap=27 * 40000)
    torch.cuda.synchronize()
    t_reg = time.perf_counter() - t0
    if a.surf_bins:
        sid = system.bodies[0]["surf"]
        nb = ctx.tune(oc.OC_TUNE_SURF_BINS, sid, 0)
        log("wall bins per axis: %d" % ctx.tune(oc.OC_TUNE_SURF_BINS, sid, max(1, int(round(nb * a.surf_bins)))))
    poses = case["poses"]
    log("warmup %d" % a.warmup)
    counts = None
    for _ in range(a.warmup):
        counts = system.step(poses)
    torch.cuda.synchronize()
    counts = system.step(poses, stats=True)
    torch.cuda.synchronize()
    st = counts.pop("stats")
    info = st["bg_cut"]

    # the plain step: default slot, eager, one chain, synchronous point
    # counts (the per-instance baseline)
    log("plain steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        counts = system.step(poses)
        torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t0) / a.steps

    # the step as served: two chains on two streams, captured once, replayed
    log("graph-replayed steps, %d timed" % a.steps)
    ss = SlotStep(system)
    ss.step(poses)
    torch.cuda.synchronize()
    same = ss.snapshot()["ib_bg"].tobytes() == system.ib_bg.cpu().numpy().tobytes()
    ss.capture()
    table = ss.pose_table_dev(poses)
    st_ = ss.stream
    for _ in range(a.warmup):
        ss.replay_table(table)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ss.replay_table(table)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms = 1e3 * t_total / a.steps
    evs = []
    for _ in range(a.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st_)
        ss.replay_table(table)
        e1.record(st_)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    lat = [x.elapsed_time(y) * 1e-3 for x, y in evs]
    snap = ss.snapshot()      # outputs of the last timed (replayed) step

    # per-kernel HIP-event timing (events on the kernel's own stream) over
    # eager launches of the same step with the two chains one after the
    # other, so that each kernel has the device to itself; then the same with
    # the chains overlapped as in the timed steps
    log("per-kernel event timing over %d steps" % a.steps)

    def kernel_times(serial):
        ctx.timing(True)
        for _ in range(a.steps):
            ss.step(poses, serial=serial)
        rep = ctx.timing_report()
        ctx.timing(False)
        return {k: dict(total_ms=v[0], launches=v[1], avg_us=1e3 * v[0] / max(v[1], 1)) for k, v in rep.items()}

    per_kernel = kernel_times(True)
    per_kernel_overlapped = kernel_times(False)

    n_pts = counts["n_bg_points"] + sum(counts["n_shell_points"])
    value = bg.n_elem / (ms / 1e3)
    # roofline of the streaming filter (HBM bound): per element the planes of
    # its FP32 box that the wavefront's early exits leave to read (at most
    # 24 B) and its iblank (1 B) written
    kf = per_kernel.get("k_filter")
    roof_filter = None
    if kf:
        bytes_per_launch = filter_bytes(bg, case["bodies"][0]["surface"].nodes, case["poses"][0])
        achieved = bytes_per_launch / (kf["avg_us"] * 1e-6) / 1e9
        roof_filter = dict(bound="hbm", kernel="k_filter", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=achieved / HBM_PEAK_GBS, traffic=measured_traffic("k_filter"),
                           algorithmic_bytes_per_launch=bytes_per_launch, avg_launch_us=kf["avg_us"])
    # the classify kernels (far/near split with ray parity, exact test, side
    # search, fringe layer) against HBM: their algorithmic bytes per launch
    # from the cut's counts; they move a few MB and are bound by the latency
    # of their dependent loads, not by bandwidth
    cls_bytes = dict(
        k_candidates=info["n_inbox"] * (8 + 24 + 1 + 4) + info["n_cand_pairs"] * 32,
        k_hit=info["n_near"] * (8 + 1 + 648) + info["n_cand_pairs"] * (32 + 216),
        k_side=info.get("n_side", 0) * (8 + 1 + 648),
        k_fringe=info["n_inbox"] * (8 + 1) + info["n_hole"] * (24 + 6))
    roof_classify = []
    for kname, nbytes in cls_bytes.items():
        kc = per_kernel.get(kname)
        if not kc:
            continue
        ach = nbytes / (kc["avg_us"] * 1e-6) / 1e9
        roof_classify.append(dict(kernel=kname, bound="latency", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                                  frac=ach / HBM_PEAK_GBS, algorithmic_bytes_per_launch=nbytes,
                                  avg_launch_us=kc["avg_us"]))
    # dominant kernel of the step; when it is the Newton kernel of the donor
    # search (FP64 VALU bound) its algorithmic FLOP per launch is
    # NEWTON_FLOP x the Newton iterations it ran
    roof = roof_filter
    dominant = max(per_kernel.items(), key=lambda kv: kv[1]["total_ms"])[0] if per_kernel else None
    kd = per_kernel.get(dominant)
    if kd and dominant == "k_dp_newton":
        iters = sum(d["n_iter"] for d in st["donor_bg"] + st["donor_shell"])
        launches_per_step = len(st["donor_bg"]) + len(st["donor_shell"])
        flop_per_launch = NEWTON_FLOP * iters / launches_per_step
        achieved = flop_per_launch / (kd["avg_us"] * 1e-6) / 1e12
        roof = dict(bound="alu", kernel=dominant, achieved=achieved, peak=FP64_VECTOR_PEAK, unit="TFLOP/s",
                    frac=achieved / FP64_VECTOR_PEAK, traffic=measured_traffic(dominant),
                    algorithmic_flop_per_launch=flop_per_launch,
                    newton_iterations_per_step=iters, avg_launch_us=kd["avg_us"])
        ko = per_kernel_overlapped.get(dominant)
        if ko:
            roof["overlapped"] = dict(avg_launch_us=ko["avg_us"],
                                      achieved=flop_per_launch / (ko["avg_us"] * 1e-6) / 1e12)
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=value, unit="elements/s", n_gpus=1, steps=a.steps, warmup=a.warmup, ms_per_step=ms,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="dimpled sphere single cut: %d^3 quadratic hexes on [-3,3]^3, 300-dimple "
                                    "R=0.5 sphere of 24576 9-node quads, 8-layer shell of 196608 hexes; cut + "
                                    "fringe + Gauss points + Newton donors in both directions" % a.bg,
                           bg_elements=bg.n_elem, surface_faces=case["bodies"][0]["surface"].n_face,
                           shell_elements=case["bodies"][0]["shell"].n_elem, parallelism="1 GPU"),
               donors_per_s=n_pts / (ms / 1e3), points_per_step=n_pts,
               latency_ms=dict(p50=1e3 * float(np.percentile(lat, 50)), p99=1e3 * float(np.percentile(lat, 99))),
               plain_ms_per_step=ms_plain, speedup_vs_plain=ms_plain / ms, slot_equals_plain=bool(same),
               cut_info=info, donor_info=dict(bg_to_shell=st["donor_bg"], shell_to_bg=st["donor_shell"]),
               registration_s=t_reg, per_kernel=per_kernel, per_kernel_overlapped=per_kernel_overlapped,
               roofline=roof, roofline_filter=roof_filter, roofline_classify=roof_classify,
               dominant_kernel=dominant)
    if roof_filter:
        ceil = copy_ceiling_gbs()
        roof_filter["copy_ceiling_gbs"] = ceil
        roof_filter["frac_of_copy_ceiling"] = roof_filter["achieved"] / ceil
    if a.serve_requests > 0:
        # the serving stream, shortened to one rate: run as a child process
        # (its own context and grid sets), so that a failure there leaves
        # this measurement standing
        log("serving stream: %d requests at %g req/s (child process)" % (a.serve_requests, a.serve_rate))
        out["serving"] = serve_child(a)
    if not a.no_cpu_baseline:
        log("oracle baseline on the host")
        cb = cpu_baseline(case, a.cpu_sample)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["precision"] = precision_report(snap, info, cb["results"])
    ctx.close()
    return out


def _percentiles(lat_s):
    return dict(p50=1e3 * float(np.percentile(lat_s, 50)), p99=1e3 * float(np.percentile(lat_s, 99)))


def run_spin(a):
    """Moving body: cold step at theta_0 = 0, then steps n = 1..N at
    R_z(2 pi n / 400), each a warm-started background re-cut (sweep bound of
    one step) plus fringe points and donors in both directions, replayed from
    two captured graphs (the two iblank parities) with device pose tables."""
    import torch
    from paper_1711_07663_amd import oc
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    from workloads import configs as CF
    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg = case["bg"]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    system = OversetSystem(ctx, case, bg_points_cap=27 * 40000)
    poses = [case["poses"][0]] + CF.spinning_poses(a.spin_steps)
    sid = system.bodies[0]["surf"]
    sweep = max(ctx.sweep_bound(sid, poses[k], poses[k + 1]) for k in range(len(poses) - 1))
    ss = SlotStep(system, warm=True, sweep=sweep)
    tables = [ss.pose_table_dev([p]) for p in poses]
    st = ss.stream

    def run_sequence(timed):
        ss.k = 0
        ss.set_poses([poses[0]])
        ss._launch(0, True)       # cold step n = 0
        ss.k = 1
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for n in range(1, len(poses)):
            if timed:
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
            ss.replay_table(tables[n])
            if timed:
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(st)
                evs.append((e0, e1))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, evs

    ss.step([poses[0]])
    torch.cuda.synchronize()
    ss.capture()
    log("warmup pass over %d steps" % a.spin_steps)
    run_sequence(False)
    log("timed pass")
    t_total, _ = run_sequence(False)
    _, evs = run_sequence(True)
    lat = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    ms = 1e3 * t_total / a.spin_steps
    # the same poses on a cold captured step (no warm start): what the warm
    # start saves at equal launch structure
    log("cold graph replays at the same poses")
    cs = SlotStep(system)
    cs.step([poses[0]])
    torch.cuda.synchronize()
    cs.capture()
    ctables = [cs.pose_table_dev([p]) for p in poses]
    for n in range(1, len(poses)):
        cs.replay_table(ctables[n])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, len(poses)):
        cs.replay_table(ctables[n])
    torch.cuda.synchronize()
    ms_cold_graph = 1e3 * (time.perf_counter() - t0) / a.spin_steps
    warm_ib = ss.ib_bg().cpu().numpy()
    cold_ib = cs.ib_bg().cpu().numpy()
    cs.close()
    # the plain per-instance GPU step: cold, eager, synchronous (default slot)
    log("plain per-step baseline")
    t0 = time.perf_counter()
    for n in range(1, len(poses)):
        system.step([poses[n]])
        torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t0) / a.spin_steps
    # per-kernel event timing over eager warm steps of the same sequence
    ctx.timing(True)
    ss.k = 0
    ss.step([poses[0]])
    for n in range(1, min(len(poses), 21)):
        ss.step([poses[n]])
    rep = ctx.timing_report()
    ctx.timing(False)
    per_kernel = {k: dict(total_ms=v[0], launches=v[1], avg_us=1e3 * v[0] / max(v[1], 1)) for k, v in rep.items()}
    cut = ss.slot.cut_info()
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=bg.n_elem / (ms / 1e3), unit="elements/s", n_gpus=1, steps=a.spin_steps, warmup=a.spin_steps,
               ms_per_step=ms, steps_per_s=1e3 / ms, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="spinning dimpled sphere: the 128^3 dimpled case rotating about z at 1 rev / "
                                    "400 steps, %d warm-started steps replayed as HIP graphs" % a.spin_steps,
                           bg_elements=bg.n_elem, sweep_bound=sweep, parallelism="1 GPU"),
               latency_ms=_percentiles(lat), plain_ms_per_step=ms_plain, speedup_vs_plain=ms_plain / ms,
               cold_graph_ms_per_step=ms_cold_graph, warm_speedup_vs_cold_graph=ms_cold_graph / ms,
               warm_equals_cold_last_step=bool(np.array_equal(warm_ib, cold_ib)),
               last_warm_cut_info=cut, per_kernel=per_kernel)
    ctx.close()
    return out


def run_ab(a):
    """The dimpled 128^3 step with the artificial-boundary receptors (Sec. 2):
    cut, AB faces of the background and of the shell, 9 flux points per face,
    donors in the other grid and 27 weights per point, both directions; the
    two-chain step replayed from its captured graph."""
    import torch
    from paper_1711_07663_amd import oc
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    from workloads import configs as CF
    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg = case["bg"]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    system = OversetSystem(ctx, case, bg_points_cap=27 * 40000, topology=a.topology)
    poses = case["poses"]
    ss = SlotStep(system, ab=True)
    # the plain step: the same launches, eager, chains one after the other,
    # waiting for each step
    for _ in range(a.warmup):
        ss.step(poses, serial=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ss.step(poses, serial=True)
        ss.stream.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t0) / a.steps
    counts = ss.counts()
    info_a, info_b = ss.slot.donor_info(), ss.slot_b.donor_info()
    ss.capture()
    table = ss.pose_table_dev(poses)
    for _ in range(a.warmup):
        ss.replay_table(table)
    torch.cuda.synchronize()
    log("graph-replayed AB steps, %d timed" % a.steps)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ss.replay_table(table)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / a.steps
    evs = []
    for _ in range(a.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ss.stream)
        ss.replay_table(table)
        e1.record(ss.stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    lat = [x.elapsed_time(y) * 1e-3 for x, y in evs]
    ctx.timing(True)
    for _ in range(a.steps):
        ss.step(poses, serial=True)
    rep = ctx.timing_report()
    ctx.timing(False)
    per_kernel = {k: dict(total_ms=v[0], launches=v[1], avg_us=1e3 * v[0] / max(v[1], 1)) for k, v in rep.items()}
    n_pts = counts["n_bg_points"] + sum(counts["n_shell_points"])
    # the weights kernel streams its output: 27 FP64 weights (216 B) written
    # and one point's donor and reference coordinates (28 B) read per point
    kw = per_kernel.get("k_interp_weights")
    roof_w = None
    if kw:
        bytes_per_launch = 244.0 * n_pts / kw["launches"] * a.steps
        achieved = bytes_per_launch / (kw["avg_us"] * 1e-6) / 1e9
        roof_w = dict(bound="hbm", kernel="k_interp_weights", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=None, algorithmic_bytes_per_launch=bytes_per_launch,
                      avg_launch_us=kw["avg_us"])
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=bg.n_elem / (ms / 1e3), unit="elements/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload="dimpled sphere, artificial-boundary receptors: %d^3 background, 24576-face "
                                    "300-dimple sphere, 8-layer shell; cut + AB faces + 3x3 Gauss flux points + "
                                    "Newton donors + 27 interpolation weights per point, both directions; the "
                                    "background cut by %s" % (a.bg, "the wall" if a.topology == "walls" else
                                                             "the shell's overset boundary"),
                           bg_elements=bg.n_elem, topology=a.topology, parallelism="1 GPU"),
               donors_per_s=n_pts / (ms / 1e3), points_per_step=n_pts, counts=counts,
               donor_info=dict(bg_to_shell=info_a, shell_to_bg=info_b),
               latency_ms=_percentiles(lat), plain_ms_per_step=ms_plain, speedup_vs_plain=ms_plain / ms,
               per_kernel=per_kernel, roofline_weights=roof_w)
    ss.close()
    ctx.close()
    return out


def run_filtered(a):
    """Ablation of the paper's truncations: the filtered cut (Sec. 4.2, Alg.
    cp0, bboxdix, cp1, cp2) of the dimpled 128^3 background against the
    exact cut, both eager and synchronous per cut."""
    import torch
    from paper_1711_07663_amd import oc
    from workloads import configs as CF
    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg, s = case["bg"], case["bodies"][0]["surface"]
    pose = case["poses"][0]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    ib_ex = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    ib = torch.empty_like(ib_ex)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / a.steps

    ms_exact = timed(lambda: ctx.cut(gid, sid, pose, ib_ex))
    ex = ib_ex.cpu().numpy()
    rows = []
    for nf1, nf2 in ((16, 4), (4, 1), (1, 1)):
        n_listed = ctx.cut_filtered(gid, [sid], pose, ib, nf1, nf2)
        ms = timed(lambda: ctx.cut_filtered(gid, [sid], pose, ib, nf1, nf2))
        got = ib.cpu().numpy()
        ctx.timing(True)
        ctx.cut_filtered(gid, [sid], pose, ib, nf1, nf2)
        rep = ctx.timing_report()
        ctx.timing(False)
        rows.append(dict(nf1=nf1, nf2=nf2, ms_per_cut=ms, elements_examined=n_listed,
                         differ_from_exact=int((got != ex).sum()),
                         holes_lost=int(((ex == 0) & (got != 0)).sum()),
                         holes_added=int(((ex != 0) & (got == 0)).sum()),
                         per_kernel={k: dict(avg_us=1e3 * v[0] / max(v[1], 1), launches=v[1])
                                     for k, v in rep.items()}))
    head = rows[0]
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=bg.n_elem / (head["ms_per_cut"] / 1e3), unit="elements/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=head["ms_per_cut"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="the paper's filtered cut (N_F^1=16, N_F^2=4) of the %d^3 dimpled-sphere "
                                    "background by its 24576-face wall, eager, one cut per step; the exact cut and "
                                    "harsher truncations beside it" % a.bg, bg_elements=bg.n_elem,
                           parallelism="1 GPU"),
               exact_ms_per_cut=ms_exact, truncations=rows)
    ctx.close()
    return out


def run_refined(a):
    """Ablation of the linearisation of the curved faces (Sec. 4.2): the
    refined cut of the dimpled 128^3 background at levels k against the
    lattice cut (oc_cut), synchronous per cut."""
    import torch
    from paper_1711_07663_amd import oc
    from workloads import configs as CF
    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg, s = case["bg"], case["bodies"][0]["surface"]
    pose = case["poses"][0]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    ib_lat = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    ib = torch.empty_like(ib_lat)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / a.steps

    ms_lat = timed(lambda: ctx.cut(gid, sid, pose, ib_lat))
    lat = ib_lat.cpu().numpy()
    rows, prev = [], None
    for k in [int(v) for v in a.levels.split(",")]:
        log("refined cut, level %d" % k)
        n_near = ctx.cut_refined(gid, [sid], pose[None], ib, k)
        ms = timed(lambda: ctx.cut_refined(gid, [sid], pose[None], ib, k))
        got = ib.cpu().numpy()
        ctx.timing(True)
        ctx.cut_refined(gid, [sid], pose[None], ib, k)
        rep = ctx.timing_report()
        ctx.timing(False)
        row = dict(k=k, ms_per_cut=ms, near_elements=n_near, sub_elements=n_near * k ** 3,
                   differ_from_lattice=int((got != lat).sum()),
                   holes_added=int(((lat != 0) & (got == 0)).sum()),
                   holes_lost=int(((lat == 0) & (got != 0)).sum()),
                   per_kernel={n: dict(avg_us=1e3 * v[0] / max(v[1], 1), launches=v[1]) for n, v in rep.items()})
        if prev is not None:
            row["differ_from_previous_level"] = int((got != prev[1]).sum())
            row["previous_level"] = prev[0]
        rows.append(row)
        prev = (k, got)
    head = rows[-1]
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=bg.n_elem / (head["ms_per_cut"] / 1e3), unit="elements/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=head["ms_per_cut"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="the refined cut (curved faces, level %d) of the %d^3 dimpled-sphere background "
                                    "by its 24576-face wall, synchronous, one cut per step; the lattice cut and "
                                    "other levels beside it" % (head["k"], a.bg), bg_elements=bg.n_elem,
                           parallelism="1 GPU"),
               lattice_ms_per_cut=ms_lat, lattice_holes=int((lat == 0).sum()), levels=rows)
    ctx.close()
    return out


def run_unblank(a):
    """Moving body with unblanking (Alg. unblank): steps n = 1..N of the
    turning, oscillating dimpled sphere.  A step is oc_unblank at the poses
    of steps n and n + 1 (two cuts in one batch, wall rule, fringe layer,
    cells to unblank; the call returns their count), then the 27 interior
    points of those cells and their donors in the shell posed at step n."""
    import torch
    from paper_1711_07663_amd import oc
    from workloads import configs as CF
    from workloads import meshes as M
    log("generating the dimpled-sphere workload")
    case = CF.dimpled(bg_n=a.bg)
    bg, body = case["bg"], case["bodies"][0]
    s, sh = body["surface"], body["shell"]
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    gid = ctx.register_grid(bg.nodes, bg.conn, bg.face_tags)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    shid = ctx.register_grid(sh.nodes, sh.conn, sh.face_tags)
    n_steps = a.spin_steps
    poses = CF.moving_poses(n_steps + 1)
    dev = torch.device("cuda", 0)
    ib = [torch.empty(bg.n_elem, dtype=torch.int8, device=dev) for _ in range(2)]
    ub = torch.empty(bg.n_elem, dtype=torch.int32, device=dev)
    cap = 27 * 20000
    pts = torch.empty((cap, 3), dtype=torch.float64, device=dev)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    donor = torch.empty(cap, dtype=torch.int32, device=dev)
    ref = torch.empty((cap, 3), dtype=torch.float64, device=dev)

    def sequence(collect):
        ctx.cut(gid, sid, poses[0], ib[0])
        torch.cuda.synchronize()
        cur = 0
        counts, orphans = [], 0
        t0 = time.perf_counter()
        for n in range(1, n_steps + 1):
            m = ctx.unblank(gid, [sid], poses[n], poses[n + 1], ib[cur], ib[1 - cur], ub)
            if m:
                if 27 * m > cap:
                    raise RuntimeError("more cells to unblank than the point buffers hold")
                ctx.element_points(gid, M.IDENTITY_POSE, ub, m, pts, src)
                ctx.donor_search(shid, poses[n], pts, 27 * m, donor, ref)
                if collect:
                    orphans += int((donor[:27 * m] < 0).sum())
            counts.append(m)
            cur = 1 - cur
        torch.cuda.synchronize()
        return time.perf_counter() - t0, counts, orphans

    log("warmup pass over %d steps" % n_steps)
    sequence(False)
    log("timed pass (eager)")
    t_total, counts, _ = sequence(False)
    _, _, orphans = sequence(True)
    ms_eager = 1e3 * t_total / n_steps

    # the same steps on a slot of their own, device pose tables, replayed
    # from the two captured parities
    from paper_1711_07663_amd.pipeline import UnblankStep
    us = UnblankStep(ctx, gid, sid, shid, ub_cap=20000)
    tables = [us.table_dev(poses[n], poses[n + 1]) for n in range(1, n_steps + 1)]

    def graph_sequence():
        us.start(poses[0])
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for n in range(1, n_steps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(us.stream)
            us.replay_table(tables[n - 1])
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record(us.stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, evs

    us.start(poses[0])
    us.step(poses[1], poses[2])
    torch.cuda.synchronize()
    us.capture()
    log("graph-replayed pass")
    graph_sequence()
    t_graph, evs = graph_sequence()
    ms = 1e3 * t_graph / n_steps
    lat = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    n_ub_last = int(us.n_ub.item())
    us.close()
    ctx.timing(True)
    sequence(False)
    rep = ctx.timing_report()
    ctx.timing(False)
    per_kernel = {k: dict(total_ms=v[0], launches=v[1], avg_us=1e3 * v[0] / max(v[1], 1)) for k, v in rep.items()}
    n_ub = int(np.sum(counts))
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=bg.n_elem / (ms / 1e3), unit="elements/s", n_gpus=1, steps=n_steps, warmup=n_steps,
               ms_per_step=ms, steps_per_s=1e3 / ms, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="unblanking of a moving body: the 128^3 dimpled case turning about z at "
                                    "1 rev / 400 steps and oscillating along x (amplitude 0.5); per step two "
                                    "cuts (t, t + dt), wall rule, fringe, cells to unblank, their interior "
                                    "points and donors in the shell; %d steps replayed as HIP graphs" % n_steps,
                           bg_elements=bg.n_elem, parallelism="1 GPU"),
               latency_ms=_percentiles(lat), eager_ms_per_step=ms_eager, speedup_vs_eager=ms_eager / ms,
               last_step_cells_unblanked=n_ub_last,
               cells_unblanked=dict(total=n_ub, max_per_step=int(np.max(counts)),
                                    steps_with_any=int(np.count_nonzero(counts))),
               interior_points=27 * n_ub, orphan_points=orphans,
               cut_elements_per_s=2 * bg.n_elem / (ms / 1e3), per_kernel=per_kernel)
    ctx.close()
    return out


def run_batch(a):
    """64 uneven instances: every instance's cut in one launch per stage
    (a slot sized for the batch, captured once as a HIP graph), against the
    plain per-instance cut (one synchronous oc_cut per instance)."""
    import torch
    from paper_1711_07663_amd import oc
    from workloads import configs as CF
    from workloads import meshes as M
    specs = CF.batch_instances(n=a.batch_n)
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    log("generating and registering %d instances" % len(specs))
    reqs, plain_args, n_tot, n_face, f_bytes = [], [], 0, 0, 0.0
    poses = torch.zeros((len(specs), 12), dtype=torch.float64, device="cuda")
    host_poses = np.stack([np.asarray(sp["pose"], dtype=np.float64) for sp in specs])
    poses.copy_(torch.from_numpy(host_poses))
    for i, sp in enumerate(specs):
        axes = (0.5, 0.35, 0.25) if sp["kind"] == "ellipsoid" else None
        bgm = M.background_grid(sp["bg_n"], -2.0, 2.0, amp=0.02)
        surf = M.cube_sphere(sp["m"], R=0.5, axes=axes, dimples=sp["dimples"], dimple_a=CF.DIMPLE_A,
                             dimple_k=CF.DIMPLE_K)
        gid = ctx.register_grid(bgm.nodes, bgm.conn)
        sid = ctx.register_cut_surface(surf.nodes, surf.conn)
        ib = torch.empty(bgm.n_elem, dtype=torch.int8, device="cuda")
        reqs.append((gid, [sid], poses[i:i + 1], ib))
        plain_args.append((gid, sid, host_poses[i], bgm.n_elem))
        n_tot += bgm.n_elem
        n_face += surf.n_face
        f_bytes += filter_bytes(bgm, surf.nodes, host_poses[i])
        del bgm, surf
    log("batch of %d instances, %d elements, %d faces" % (len(specs), n_tot, n_face))
    # eager batches on the default slot, before and after autotuning
    from paper_1711_07663_amd import autotune
    host_reqs = [(g_, s_, host_poses[i:i + 1], ib_) for i, (g_, s_, _, ib_) in enumerate(reqs)]
    surf_faces = {}
    for (gid, sids, _, _), sp in zip(reqs, specs):
        surf_faces[sids[0]] = 6 * sp["m"] * sp["m"]
    t_untuned = autotune._time(lambda: ctx.cut_batch(host_reqs), 3)
    t0 = time.perf_counter()
    params, tune_report = autotune.tune_batch(ctx, host_reqs, surf_faces)
    t_tune = time.perf_counter() - t0
    t_tuned = autotune._time(lambda: ctx.cut_batch(host_reqs), 3)
    log("autotuned in %.1f s: %s (eager batch %.2f -> %.2f ms)" % (t_tune, params, 1e3 * t_untuned, 1e3 * t_tuned))
    slot = ctx.create_batch_slot(reqs)
    for _ in range(a.warmup):
        slot.cut_batch(reqs)
    torch.cuda.synchronize()
    info = slot.cut_info()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        slot.set_stream(torch.cuda.current_stream())
        slot.cut_batch(reqs)
    slot.set_stream(slot.stream)
    st = slot.stream
    lat = []
    with torch.cuda.stream(st):
        for _ in range(a.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            g.replay()
            e1.record(st)
            lat.append((e0, e1))
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / a.steps
    lat = [x.elapsed_time(y) * 1e-3 for x, y in lat]
    batch_out = [r[3].clone() for r in reqs]
    # plain: one synchronous cut per instance on the default slot
    plain_ib = [torch.empty_like(r[3]) for r in reqs]
    for (gid, sid, pz, ne), ib in zip(plain_args, plain_ib):
        ctx.cut(gid, sid, pz, ib)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, a.steps // 4)):
        for (gid, sid, pz, ne), ib in zip(plain_args, plain_ib):
            ctx.cut(gid, sid, pz, ib)
            torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / max(1, a.steps // 4)
    same = all(torch.equal(x, y) for x, y in zip(batch_out, plain_ib))
    # the cut service: every instance submitted back to back (oc_submit) and
    # then waited for; requests run on service slots of their own streams
    svc_ib = [torch.empty_like(r[3]) for r in reqs]

    def serve_all():
        tickets = [ctx.submit(gid, [sid], pz.reshape(1, 12), ib)
                   for (gid, sid, pz, ne), ib in zip(plain_args, svc_ib)]
        for t in tickets:
            ctx.wait(t)

    serve_all()     # creates the service slots
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, a.steps // 4)):
        serve_all()
    t_service = (time.perf_counter() - t0) / max(1, a.steps // 4)
    svc_info = ctx.service_info()
    svc_same = all(torch.equal(x, y) for x, y in zip(svc_ib, plain_ib))
    log("service: %.2f ms for %d requests on %d slots (peak %d running)" % (
        1e3 * t_service, len(reqs), svc_info["slots"], svc_info["peak_running"]))
    # per-kernel event timing of eager batch launches
    ctx.timing(True)
    for _ in range(5):
        slot.cut_batch(reqs)
    rep = ctx.timing_report()
    ctx.timing(False)
    per_kernel = {k: dict(total_ms=v[0], launches=v[1], avg_us=1e3 * v[0] / max(v[1], 1)) for k, v in rep.items()}
    kf = per_kernel.get("k_filter")
    roof = None
    if kf:
        achieved = f_bytes / (kf["avg_us"] * 1e-6) / 1e9
        roof = dict(bound="hbm", kernel="k_filter", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None, algorithmic_bytes_per_launch=f_bytes,
                    avg_launch_us=kf["avg_us"])
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=n_tot / t_batch, unit="elements/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=1e3 * t_batch, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload="64 uneven instances from SeedSequence(1711): backgrounds 16^3..96^3 on "
                                    "[-2,2]^3, sphere / ellipsoid / dimpled bodies of 6 m^2 faces (m 8..64), "
                                    "random rotation and +-0.3 translation; cut only, one graph-captured batch",
                           instances=len(specs), total_elements=n_tot, total_faces=n_face, parallelism="1 GPU"),
               latency_ms=_percentiles(lat), plain_ms=1e3 * t_plain, plain_elements_per_s=n_tot / t_plain,
               speedup_vs_plain=t_plain / t_batch, batch_equals_plain=bool(same), cut_info=info,
               service=dict(ms=1e3 * t_service, elements_per_s=n_tot / t_service, equals_plain=bool(svc_same),
                            slots=svc_info["slots"], peak_running=svc_info["peak_running"],
                            slot_gb=svc_info["slot_bytes"] / (1 << 30)),
               autotune=dict(params=params, report=tune_report, seconds=t_tune, eager_ms_untuned=1e3 * t_untuned,
                             eager_ms_tuned=1e3 * t_tuned),
               per_kernel=per_kernel, roofline=roof,
               instance_sizes=[(sp["bg_n"], sp["m"], sp["kind"]) for sp in specs])
    slot.close()
    ctx.close()
    return out


def serving_systems(ctx, dimpled=None):
    """The four grid sets of the serving stream, registered on ctx: the tiny
    case, the dimpled 128^3 case (whose spinning poses give the moving-ball
    set), and the two-body case on a 160^3 background.  ``dimpled``: an
    (case, OversetSystem) pair already registered on ctx, reused."""
    from paper_1711_07663_amd.pipeline import OversetSystem
    from workloads import configs as CF
    tiny, two = CF.tiny(), CF.two_body()
    if dimpled is None:
        dimp = CF.dimpled()
        dsys = OversetSystem(ctx, dimp, bg_points_cap=27 * 40000)
    else:
        dimp, dsys = dimpled
    systems = dict(tiny=OversetSystem(ctx, tiny), dimpled=dsys,
                   two_body=OversetSystem(ctx, two, bg_points_cap=27 * 80000))
    return systems, dict(tiny=tiny, dimpled=dimp, two_body=two)


def serve_stream(ctx, systems, cases, rates, n_requests, budget_gb, seed=7663):
    """Poisson arrivals (seed) at each rate, each request one of the four
    sets drawn uniformly (the spinning ball and the two-body case at a
    random step), served with continuous batching (Server) and, on the same
    arrival trace, one request at a time on the default slot.  Returns the
    per-rate results and the server."""
    import torch
    from paper_1711_07663_amd.serve import Server
    from workloads import configs as CF
    sets = ["tiny", "dimpled", "spin", "two_body"]
    rng = np.random.default_rng(seed)

    def draw():
        k = sets[int(rng.integers(0, 4))]
        if k == "tiny":
            return "tiny", cases["tiny"]["poses"]
        if k == "dimpled":
            return "dimpled", cases["dimpled"]["poses"]
        n = int(rng.integers(1, 201))
        if k == "spin":
            return "dimpled", [CF.spinning_poses(n)[-1]]
        return "two_body", CF.two_body_poses(n)

    budget = int(budget_gb * (1 << 30))
    srv = Server(ctx, systems, budget, max_slots=16)
    log("warming slots")
    for _ in range(3):
        for name in systems:
            for _ in range(2):
                srv.submit(name, cases[name]["poses"])
        srv.drain()
    torch.cuda.synchronize()
    results = []
    for lam in rates:
        gaps = rng.exponential(1.0 / lam, size=n_requests)
        arrivals = np.cumsum(gaps)
        reqs = [draw() for _ in range(n_requests)]
        for mode in ("served", "one_at_a_time"):
            log("rate %g req/s, %s, %d requests" % (lam, mode, n_requests))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat = []
            if mode == "served":
                srv.done = []
                i = 0
                while i < n_requests or srv.queue or srv.busy:
                    now = time.perf_counter() - t0
                    while i < n_requests and arrivals[i] <= now:
                        srv.submit(reqs[i][0], reqs[i][1], t_arrival=t0 + arrivals[i])
                        i += 1
                    srv.pump()
                lat = [r["t_done"] - r["t_arrival"] for r in srv.done]
                t_end = max(r["t_done"] for r in srv.done) - t0
            else:
                for i in range(n_requests):
                    now = time.perf_counter() - t0
                    if arrivals[i] > now:
                        time.sleep(max(0.0, arrivals[i] - now - 2e-4))
                        while time.perf_counter() - t0 < arrivals[i]:
                            pass
                    systems[reqs[i][0]].step(reqs[i][1])
                    torch.cuda.synchronize()
                    lat.append(time.perf_counter() - t0 - arrivals[i])
                t_end = time.perf_counter() - t0
            results.append(dict(rate=lam, mode=mode, requests=n_requests, throughput=n_requests / t_end,
                                latency_ms=_percentiles(lat), mean_ms=1e3 * float(np.mean(lat)),
                                slots=len(srv.slots) if mode == "served" else 1))
    return results, srv


def serve_child(a):
    """bench.py --workload serve at one rate in a child process; its results,
    or the child's failure."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "serve", "--rates", "%g" % a.serve_rate,
           "--requests", str(a.serve_requests), "--budget-gb", "%g" % a.budget_gb]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    for line in r.stderr.splitlines():
        print(line, file=sys.stderr, flush=True)
    lines = [x for x in r.stdout.splitlines() if x.startswith("{")]
    if r.returncode != 0 or not lines:
        return dict(error="serving child exited with status %d" % r.returncode)
    res = json.loads(lines[-1])
    sv = {x["mode"]: x for x in res["rates"]}
    return dict(rate_per_s=a.serve_rate, requests=a.serve_requests,
                sets="tiny 16^3, dimpled 128^3, spinning ball at a random step, two-body 160^3 at a random step",
                served=dict(p50_ms=sv["served"]["latency_ms"]["p50"], p99_ms=sv["served"]["latency_ms"]["p99"],
                            throughput_per_s=sv["served"]["throughput"], slots=sv["served"]["slots"]),
                one_at_a_time=dict(p50_ms=sv["one_at_a_time"]["latency_ms"]["p50"],
                                   p99_ms=sv["one_at_a_time"]["latency_ms"]["p99"],
                                   throughput_per_s=sv["one_at_a_time"]["throughput"]),
                hbm_used_gb=res.get("hbm_used_gb"))


def run_serve(a):
    """Poisson arrivals over four grid sets (tiny case, dimpled case, the
    spinning ball at a random step, the two-body case on a 160^3 background
    at a random step), served with continuous batching (slots on their own
    streams, graph replays, admission by HBM budget), against one-at-a-time
    service of the same arrival trace on the default slot."""
    import torch
    from paper_1711_07663_amd import oc
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    log("registering the grid sets")
    systems, cases = serving_systems(ctx)
    results, srv = serve_stream(ctx, systems, cases, [float(x) for x in a.rates.split(",")], a.requests,
                                a.budget_gb)
    served = [r for r in results if r["mode"] == "served"]
    best = max(served, key=lambda r: r["rate"])
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=best["throughput"], unit="requests/s", n_gpus=1, steps=a.requests, warmup=6,
               ms_per_step=1e3 / best["throughput"], higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="serving: Poisson arrivals at %s req/s over {tiny 16^3 case, dimpled 128^3 "
                                    "case, spinning ball at a random step, two-body 160^3 case at a random step}, "
                                    "continuous batching with slots admitted under a %.0f GB budget"
                                    % (a.rates, a.budget_gb), parallelism="1 GPU"),
               latency_ms=best["latency_ms"], rates=results, slots=len(srv.slots),
               hbm_used_gb=srv.used_bytes() / (1 << 30), refused_admissions=srv.n_refused)
    ctx.close()
    return out


def run_service(a):
    """Cut requests served as they arrive by the native cut service
    (oc_submit / oc_wait): Poisson arrivals (seed 7663) at the given rates,
    each request one of the 64 uneven instances drawn uniformly, against the
    same arrival trace served one synchronous cut at a time."""
    import torch
    from paper_1711_07663_amd import oc
    from workloads import configs as CF
    from workloads import meshes as M
    specs = CF.batch_instances(n=a.batch_n)
    torch.cuda.set_device(0)
    ctx = oc.Context(device=0)
    log("registering %d instances" % len(specs))
    inst = []
    for sp in specs:
        axes = (0.5, 0.35, 0.25) if sp["kind"] == "ellipsoid" else None
        bgm = M.background_grid(sp["bg_n"], -2.0, 2.0, amp=0.02)
        surf = M.cube_sphere(sp["m"], R=0.5, axes=axes, dimples=sp["dimples"], dimple_a=CF.DIMPLE_A,
                             dimple_k=CF.DIMPLE_K)
        gid = ctx.register_grid(bgm.nodes, bgm.conn)
        sid = ctx.register_cut_surface(surf.nodes, surf.conn)
        pose = np.asarray(sp["pose"], dtype=np.float64)
        # a few outputs per instance, so that repeated requests of one
        # instance can be in flight together
        bufs = [torch.empty(bgm.n_elem, dtype=torch.int8, device="cuda") for _ in range(4)]
        inst.append(dict(gid=gid, sid=sid, pose=pose, bufs=bufs, busy=[None] * 4, next=0))
        del bgm, surf
    solo = [torch.empty_like(d["bufs"][0]) for d in inst]
    log("warming the service and the plain path")
    for d, o in zip(inst, solo):
        assert ctx.wait(ctx.submit(d["gid"], [d["sid"]], d["pose"].reshape(1, 12), d["bufs"][0]))
        ctx.cut(d["gid"], d["sid"], d["pose"], o)
    torch.cuda.synchronize()
    same = all(torch.equal(d["bufs"][0], o) for d, o in zip(inst, solo))
    rng = np.random.default_rng(7663)
    rates = [float(x) for x in a.service_rates.split(",")]
    results = []
    for lam in rates:
        n_req = a.requests
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
        which = rng.integers(0, len(inst), size=n_req)
        for mode in ("service", "one_at_a_time"):
            log("rate %g req/s, %s, %d requests" % (lam, mode, n_req))
            torch.cuda.synchronize()
            lat = []
            t0 = time.perf_counter()
            if mode == "service":
                pending = []   # (ticket, arrival, instance, buffer)
                i = 0
                while i < n_req or pending:
                    now = time.perf_counter() - t0
                    while i < n_req and arrivals[i] <= now:
                        d = inst[which[i]]
                        k = d["next"]
                        d["next"] = (k + 1) % len(d["bufs"])
                        if d["busy"][k] is not None:   # that output is still in flight: wait for it
                            t_old, a_old = d["busy"][k]
                            ctx.wait(t_old)
                            lat.append(time.perf_counter() - t0 - a_old)
                            pending = [p for p in pending if p[0] != t_old]
                        t = ctx.submit(d["gid"], [d["sid"]], d["pose"].reshape(1, 12), d["bufs"][k])
                        d["busy"][k] = (t, arrivals[i])
                        pending.append((t, arrivals[i], which[i], k))
                        i += 1
                    still = []
                    for t, arr, w, k in pending:
                        if ctx.wait(t, 0):
                            lat.append(time.perf_counter() - t0 - arr)
                            inst[w]["busy"][k] = None
                        else:
                            still.append((t, arr, w, k))
                    pending = still
                t_end = time.perf_counter() - t0
            else:
                for i in range(n_req):
                    now = time.perf_counter() - t0
                    if arrivals[i] > now:
                        time.sleep(max(0.0, arrivals[i] - now - 2e-4))
                        while time.perf_counter() - t0 < arrivals[i]:
                            pass
                    d = inst[which[i]]
                    ctx.cut(d["gid"], d["sid"], d["pose"], solo[which[i]])
                    torch.cuda.synchronize()
                    lat.append(time.perf_counter() - t0 - arrivals[i])
                t_end = time.perf_counter() - t0
            results.append(dict(rate=lam, mode=mode, requests=n_req, throughput=n_req / t_end,
                                latency_ms=_percentiles(lat), mean_ms=1e3 * float(np.mean(lat))))
    info = ctx.service_info()
    served = [r for r in results if r["mode"] == "service"]
    best = max(served, key=lambda r: r["rate"])
    out = dict(metric="elements cut+classified/s and donors/s per step; p50/p99 connectivity latency",
               value=best["throughput"], unit="requests/s", n_gpus=1, steps=a.requests, warmup=len(inst),
               ms_per_step=1e3 / best["throughput"], higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="native cut service: Poisson arrivals at %s req/s, each request one of the 64 "
                                    "uneven instances (backgrounds 16^3..96^3, surfaces of 6 m^2 faces, m 8..64), "
                                    "oc_submit / oc_wait" % a.service_rates, parallelism="1 GPU"),
               latency_ms=best["latency_ms"], rates=results, service_equals_plain=bool(same),
               service=dict(slots=info["slots"], peak_running=info["peak_running"],
                            slot_gb=info["slot_bytes"] / (1 << 30)))
    ctx.close()
    return out


if __name__ == "__main__":
    main()
