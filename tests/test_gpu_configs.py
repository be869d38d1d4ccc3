"""Oracle parity of the paths the benchmark workloads run, at their sizes.

* the dimpled 128^3 step as bench.py times it: a SlotStep captured once and
  replayed from a device pose table (two chains on two streams);
* the spinning body at full size: warm-started graph replays over three
  consecutive poses;
* a batch with the real size classes of the 64-instance workload (its
  largest instances and a 96^3 background cut by a 24 576-face dimpled
  sphere), long enough a side list that the one-wavefront-per-item side
  search runs;
* served requests (continuous batching over slots) including a 160^3
  two-body request, each against the oracle;
* a donor search whose pairs overflow the pair capacity (the one-candidate-
  at-a-time path), and a cut at |x| ~ 1e3.

Large cuts are compared by the band method (parity_util.band_hole_mask);
every receptor point and donor is compared.  Bar: iblank and donor ids
bit-exact, reference coordinates within 1e-10, points within 1e-12."""
import sys
import time

import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M

import parity_util as PU

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def _ctx():
    import torch
    from paper_1711_07663_amd import oc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return oc.Context(device=0)


def test_replayed_step_full_size(orc):
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("dimpled 128^3: the benchmark's replayed two-chain step")
    case = CF.dimpled()
    ctx = _ctx()
    try:
        system = OversetSystem(ctx, case, bg_points_cap=27 * 40000)
        ss = SlotStep(system)
        ss.step(case["poses"])
        torch.cuda.synchronize()
        ss.capture()
        table = ss.pose_table_dev(case["poses"])
        for _ in range(3):
            ss.replay_table(table)
        got = ss.snapshot()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    t0 = time.time()
    want = PU.oracle_step_band(case, case["poses"])
    _note("oracle step in %.1f s" % (time.time() - t0))
    PU.compare(got, want)
    assert (got["ib_bg"] == 0).sum() > 6000


def test_spinning_full_size_warm(orc):
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("spinning dimpled sphere at 128^3: warm-started graph replays")
    case = CF.dimpled()
    ctx = _ctx()
    poses = [M.IDENTITY_POSE] + CF.spinning_poses(3)
    snaps = []
    try:
        system = OversetSystem(ctx, case, bg_points_cap=27 * 40000)
        sweep = ctx.sweep_bound(system.bodies[0]["surf"], poses[0], poses[1])
        ss = SlotStep(system, warm=True, sweep=sweep)
        ss.step([poses[0]])
        torch.cuda.synchronize()
        ss.capture()
        for p in poses[1:]:
            ss.replay([p])
            snaps.append(ss.snapshot())
        assert ss.cold_fallbacks == 0
    finally:
        torch.cuda.synchronize()
        ctx.close()
    for n, (p, got) in enumerate(zip(poses[1:], snaps), start=1):
        _note("spinning step %d against the oracle" % n)
        PU.compare(got, PU.oracle_step_band(case, [p]))


def _batch_specs():
    specs = CF.batch_instances()
    big = sorted(specs, key=lambda s: -s["bg_n"] ** 3)[:5]
    small = [specs[i] for i in (3, 17, 40, 54)]
    rng = np.random.default_rng(9664)
    extra = dict(index=64, bg_n=96, m=64, kind="dimpled", dimples=300, pose=M.random_pose(rng, 0.3))
    return big + small + [extra]


def test_batch_real_size_classes(orc):
    import torch
    _note("batch of the workload's size classes (96^3 x 24 576 faces included)")
    specs = _batch_specs()
    ctx = _ctx()
    cases, outs = [], []
    try:
        reqs = []
        for sp in specs:
            axes = (0.5, 0.35, 0.25) if sp["kind"] == "ellipsoid" else None
            bg = M.background_grid(sp["bg_n"], -2.0, 2.0, amp=0.02)
            s = M.cube_sphere(sp["m"], R=0.5, axes=axes, dimples=sp["dimples"], dimple_a=CF.DIMPLE_A,
                              dimple_k=CF.DIMPLE_K)
            gid = ctx.register_grid(bg.nodes, bg.conn)
            sid = ctx.register_cut_surface(s.nodes, s.conn)
            ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
            pose = np.asarray(sp["pose"], dtype=np.float64)
            reqs.append((gid, [sid], pose.reshape(1, 12), ib))
            cases.append((bg, s, pose))
            outs.append(ib)
        ctx.cut_batch(reqs)
        info = ctx.last_cut_info()
        got = [ib.cpu().numpy() for ib in outs]
    finally:
        torch.cuda.synchronize()
        ctx.close()
    _note("batch cut info %s" % info)
    assert info["n_side"] > 512, "the long side list (one wavefront per item) must be reached"
    for sp, (bg, s, pose), g in zip(specs, cases, got):
        want = PU.band_cut(bg, [s], [pose])
        bad = np.nonzero(g != want)[0]
        assert bad.size == 0, "instance %d (%d^3, m %d): %d elements differ, first %s" % (
            sp["index"], sp["bg_n"], sp["m"], bad.size, bad[:8])


def test_served_requests_match_oracle(orc):
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem
    from paper_1711_07663_amd.serve import Server
    _note("served requests (tiny, dimpled 128^3, two-body 160^3) against the oracle")
    tiny, dimp, two = CF.tiny(), CF.dimpled(), CF.two_body()
    ctx = _ctx()
    results = {}

    def done(req, ss):
        results[req["tag"]] = ss.snapshot()

    reqs = [("tiny", tiny["poses"], tiny), ("dimpled", [CF.spinning_poses(57)[-1]], dimp),
            ("two_body", CF.two_body_poses(37), two), ("tiny", [M.pose_rz(0.4, (0.05, 0.0, -0.02))], tiny),
            ("two_body", CF.two_body_poses(0), two)]
    try:
        systems = dict(tiny=OversetSystem(ctx, tiny), dimpled=OversetSystem(ctx, dimp, bg_points_cap=27 * 40000),
                       two_body=OversetSystem(ctx, two, bg_points_cap=27 * 80000))
        srv = Server(ctx, systems, 64 << 30, max_slots=8, on_done=done)
        for i, (name, poses, _) in enumerate(reqs):
            srv.submit(name, poses, tag=i)
        srv.drain()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    for i, (name, poses, case) in enumerate(reqs):
        _note("request %d (%s) against the oracle" % (i, name))
        PU.compare(results[i], PU.oracle_step_band(case, poses))


def test_pair_overflow_matches_oracle(orc):
    """Pairs beyond the capacity (a small cap set by OC_TUNE_DONOR_PAIRS):
    those points are solved one candidate at a time in ascending id."""
    import torch
    from paper_1711_07663_amd import oc
    _note("donor search with the pair capacity capped at 3000 pairs")
    case = CF.dimpled(bg_n=40, m=16, layers=2, dimples=60)
    bg, sh = case["bg"], case["bodies"][0]["shell"]
    ctx = _ctx()
    try:
        gid = ctx.register_grid(bg.nodes, bg.conn)
        pts = orc.fringe_points(sh, orc.fringe_elements(orc.cut(sh, [], [])), M.pose_rz(0.2))
        n = pts.shape[0]
        p = torch.from_numpy(pts).cuda()
        d = torch.empty(n, dtype=torch.int32, device="cuda")
        r = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        assert ctx.tune(oc.OC_TUNE_DONOR_PAIRS, 0, 3000) == 3000
        ctx.donor_search(gid, M.IDENTITY_POSE, p, n, d, r)
        info = ctx.last_donor_info()
        d_g, r_g = d.cpu().numpy(), r.cpu().numpy()
        ctx.tune(oc.OC_TUNE_DONOR_PAIRS, 0, 0)
        ctx.donor_search(gid, M.IDENTITY_POSE, p, n, d, r)
        info0 = ctx.last_donor_info()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    _note("overflow points %d of %d (uncapped: %d)" % (info["n_overflow"], n, info0["n_overflow"]))
    assert info["n_overflow"] > n // 2 and info0["n_overflow"] == 0
    d_o, r_o, _ = orc.donor_search(bg, pts)
    assert np.array_equal(d_g, d_o)
    ok = d_o >= 0
    assert np.abs(r_g[ok] - r_o[ok]).max() <= PU.XI_TOL
    assert np.all(np.isnan(r_g[~ok]))


def test_cut_far_from_origin(orc):
    """The tiny case moved to about (1000, 1000, 1000), where the FP32 box
    filter's 2^-20 max|x| inflation term is what keeps every close pair."""
    import torch
    from test_filter_bound import far_tiny
    _note("tiny case at |x| ~ 1e3")
    bg, s, pose = far_tiny()
    ctx = _ctx()
    try:
        gid = ctx.register_grid(bg.nodes, bg.conn)
        sid = ctx.register_cut_surface(s.nodes, s.conn)
        ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        ctx.cut(gid, sid, pose, ib)
        got = ib.cpu().numpy()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    want = orc.cut(bg, [s], [pose])
    assert np.array_equal(got, want)
    assert (want == orc.HOLE).sum() > 50


def test_side_list_and_bin_walk_agree(orc):
    """The tie stage of the side search reads the faces its wavefronts listed
    in the second stage; with the lists capped at one face
    (OC_TUNE_SIDE_LIST) an element with more faces within its bound walks the
    bins again.  Both give the oracle's iblank."""
    import torch
    from paper_1711_07663_amd import oc
    _note("side search: face lists against the bin walk (48^3, m 16, 60 dimples)")
    bg = M.background_grid(48, -1.2, 1.2, amp=0.02)
    s = M.cube_sphere(16, R=0.5, dimples=60, dimple_a=CF.DIMPLE_A, dimple_k=CF.DIMPLE_K)
    pose = np.asarray(M.random_pose(np.random.default_rng(4471), 0.2), dtype=np.float64)
    ctx = _ctx()
    got, infos = {}, {}
    try:
        gid = ctx.register_grid(bg.nodes, bg.conn)
        sid = ctx.register_cut_surface(s.nodes, s.conn)
        for cap in (1, 0):
            assert ctx.tune(oc.OC_TUNE_SIDE_LIST, 0, cap) == (cap or 64)
            ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
            ctx.cut_batch([(gid, [sid], pose.reshape(1, 12), ib)])
            infos[cap] = ctx.last_cut_info()
            got[cap] = ib.cpu().numpy()
        assert ctx.tune(oc.OC_TUNE_SIDE_LIST, 0, -1) == 64
    finally:
        torch.cuda.synchronize()
        ctx.close()
    _note("cut info %s" % infos[0])
    assert infos[0]["n_side"] > 0, "the side search must run on this case"
    want = PU.band_cut(bg, [s], [pose])
    for cap in (1, 0):
        bad = np.nonzero(got[cap] != want)[0]
        assert bad.size == 0, "side list cap %d: %d elements differ, first %s" % (cap, bad.size, bad[:8])
