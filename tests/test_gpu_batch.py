"""Batched cuts: many uneven (grid, surfaces, pose) requests in one launch per
stage give, request by request, the iblank of the request cut alone, and the
oracle's."""
import sys

import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1711_07663_amd import oc
    c = oc.Context(device=0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _small_batch(n=8):
    """Uneven small instances drawn like the 64-instance batch (same
    generator, smaller size ranges)."""
    specs = CF.batch_instances(n=n, n_lo=8, n_hi=22, m_lo=3, m_hi=8)
    return [CF.batch_case(s, layers=2) for s in specs]


def _register(ctx, cases):
    out = []
    for c in cases:
        gid = ctx.register_grid(c["bg"].nodes, c["bg"].conn)
        sid = ctx.register_cut_surface(c["bodies"][0]["surface"].nodes, c["bodies"][0]["surface"].conn)
        out.append((gid, sid))
    return out


def test_batch_equals_solo_and_oracle(ctx, orc):
    import torch
    _note("batch of 8 uneven instances vs solo cuts vs oracle")
    cases = _small_batch(8)
    ids = _register(ctx, cases)
    outs = [torch.full((c["bg"].n_elem,), 7, dtype=torch.int8, device="cuda") for c in cases]
    reqs = [(g, [s], c["poses"][0].reshape(1, 12), ib) for (g, s), c, ib in zip(ids, cases, outs)]
    ctx.cut_batch(reqs)
    torch.cuda.synchronize()
    info = ctx.last_cut_info()
    assert info["n_elem"] == sum(c["bg"].n_elem for c in cases)
    solo = torch.empty(max(c["bg"].n_elem for c in cases), dtype=torch.int8, device="cuda")
    n_hole = 0
    for (g, s), c, ib in zip(ids, cases, outs):
        ctx.cut(g, s, c["poses"][0], solo[:c["bg"].n_elem])
        torch.cuda.synchronize()
        got = ib.cpu().numpy()
        assert np.array_equal(got, solo[:c["bg"].n_elem].cpu().numpy())
        ref = orc.cut(c["bg"], [c["bodies"][0]["surface"]], c["poses"])
        assert np.array_equal(got, ref), c["name"]
        n_hole += int((got == 0).sum())
    assert n_hole > 0
    # batch statistics: holes of every output, item statuses
    assert info["n_hole"] == n_hole
    assert 0 < info["n_hit"] <= info["n_near"] <= info["n_inbox"]
    assert info["n_near"] + info["n_far"] <= info["n_inbox"]
    assert info["n_cand_pairs"] >= info["n_near"]


def test_batch_mixed_requests(ctx, orc):
    """Union of two surfaces, a request with no surface (overset faces only),
    one surface used by two requests at different poses, and a singleton."""
    import torch
    _note("mixed batch: union, no-surface, shared surface")
    bg = M.background_grid(18, -1.5, 1.5, amp=0.02)
    s1 = M.cube_sphere(5, R=0.4, dimples=12, dimple_a=0.07, dimple_k=0.015)
    s2 = M.cube_sphere(4, R=0.3, axes=(0.3, 0.22, 0.18))
    sh = M.shell_grid(s1, 2, r_out=0.8)
    g = ctx.register_grid(bg.nodes, bg.conn)
    gs = ctx.register_grid(sh.nodes, sh.conn, sh.face_tags)
    a = ctx.register_cut_surface(s1.nodes, s1.conn)
    b = ctx.register_cut_surface(s2.nodes, s2.conn)
    pa = M.pose_rz(0.3, (-0.45, 0.1, 0.0))
    pb = M.pose_rz(-0.7, (0.55, -0.05, 0.1))
    pc = M.random_pose(np.random.default_rng(3), 0.3)
    o = [torch.empty(bg.n_elem, dtype=torch.int8, device="cuda") for _ in range(3)]
    o_sh = torch.empty(sh.n_elem, dtype=torch.int8, device="cuda")
    reqs = [(g, [a, b], np.stack([pa, pb]), o[0]),
            (gs, [], None, o_sh),
            (g, [a], pc.reshape(1, 12), o[1]),
            (g, [b], pa.reshape(1, 12), o[2])]
    ctx.cut_batch(reqs)
    torch.cuda.synchronize()
    assert np.array_equal(o[0].cpu().numpy(), orc.cut(bg, [s1, s2], [pa, pb]))
    assert np.array_equal(o_sh.cpu().numpy(), orc.cut(sh, [], []))
    assert np.array_equal(o[1].cpu().numpy(), orc.cut(bg, [s1], [pc]))
    assert np.array_equal(o[2].cpu().numpy(), orc.cut(bg, [s2], [pa]))


def test_batch_slot_graph_replay(ctx):
    """A batch on a slot sized by oc_slot_create_batch, captured once and
    replayed with new device poses; every replay equals the eager batch."""
    import torch
    _note("batch slot: eager vs graph replay, 3 pose sets")
    cases = _small_batch(5)
    ids = _register(ctx, cases)
    outs = [torch.empty(c["bg"].n_elem, dtype=torch.int8, device="cuda") for c in cases]
    poses = torch.zeros((len(cases), 12), dtype=torch.float64, device="cuda")
    reqs = [(g, [s], poses[i:i + 1], outs[i]) for i, (g, s) in enumerate(ids)]
    slot = ctx.create_batch_slot(reqs)
    rng = np.random.default_rng(11)
    sets = [np.stack([M.random_pose(rng, 0.3) for _ in cases]) for _ in range(3)]

    def run_eager(P):
        with torch.cuda.stream(slot.stream):
            poses.copy_(torch.from_numpy(P))
        slot.cut_batch(reqs)
        torch.cuda.synchronize()
        return [o.cpu().numpy().copy() for o in outs]

    eager = [run_eager(P) for P in sets]
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        slot.set_stream(torch.cuda.current_stream())
        slot.cut_batch(reqs)
    slot.set_stream(slot.stream)
    for k in (2, 0, 1, 2):
        poses.copy_(torch.from_numpy(sets[k]))
        torch.cuda.synchronize()
        for o in outs:
            o.fill_(9)
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager[k], outs):
            assert np.array_equal(a, b.cpu().numpy())
    # the slot refuses a larger batch
    from paper_1711_07663_amd import oc
    with pytest.raises(oc.OcError):
        slot.cut_batch(reqs + reqs[:1])
    slot.close()


def test_batch_errors(ctx):
    import torch
    from paper_1711_07663_amd import oc
    _note("batch argument errors")
    bg = M.background_grid(6, -1, 1)
    s = M.cube_sphere(2, R=0.4)
    g = ctx.register_grid(bg.nodes, bg.conn)
    a = ctx.register_cut_surface(s.nodes, s.conn)
    ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    with pytest.raises(oc.OcError) as e:
        ctx.cut_batch([(g, [a], M.IDENTITY_POSE.reshape(1, 12), ib), (g, [a], M.IDENTITY_POSE.reshape(1, 12), ib)])
    assert e.value.status == oc.OC_EINVAL
    with pytest.raises(oc.OcError) as e:
        ctx.cut_batch([(g, [999], M.IDENTITY_POSE.reshape(1, 12), ib)])
    assert e.value.status == oc.OC_ENOTFOUND
    bad = M.IDENTITY_POSE.copy()
    bad[3] = np.nan
    with pytest.raises(oc.OcError) as e:
        ctx.cut_batch([(g, [a], bad.reshape(1, 12), ib)])
    assert e.value.status == oc.OC_EINVAL
    ctx.cut_batch([])


def test_tuning_knobs_do_not_change_results(ctx, tmp_path):
    """Bin caps and exact-stage wavefront counts change speed only."""
    import torch
    from paper_1711_07663_amd import autotune, oc
    _note("tuning knobs: same iblank under every setting")
    cases = _small_batch(6)
    ids = _register(ctx, cases)
    outs = [torch.empty(c["bg"].n_elem, dtype=torch.int8, device="cuda") for c in cases]
    reqs = [(g, [s], c["poses"][0].reshape(1, 12), ib) for (g, s), c, ib in zip(ids, cases, outs)]
    ctx.cut_batch(reqs)
    torch.cuda.synchronize()
    ref = [o.cpu().numpy().copy() for o in outs]
    auto = {s: ctx.tune(oc.OC_TUNE_SURF_BINS, s, 0) for _, s in ids}
    for factor, waves in ((0.5, 64), (0.25, 1), (1.0, 20000), (0.01, 8192)):
        for s, nb in auto.items():
            assert ctx.tune(oc.OC_TUNE_SURF_BINS, s, max(1, int(nb * factor))) >= 1
        ctx.tune(oc.OC_TUNE_EXACT_WAVES, 0, waves)
        for o in outs:
            o.fill_(5)
        ctx.cut_batch(reqs)
        torch.cuda.synchronize()
        for a, b in zip(ref, outs):
            assert np.array_equal(a, b.cpu().numpy())
    faces = {s: c["bodies"][0]["surface"].n_face for (g, s), c in zip(ids, cases)}
    params, report = autotune.tune_batch(ctx, reqs, faces, reps=1)
    assert params["exact_waves"] in (2048, 4096, 8192, 16384)
    ctx.cut_batch(reqs)
    torch.cuda.synchronize()
    for a, b in zip(ref, outs):
        assert np.array_equal(a, b.cpu().numpy())
    assert params["filter_block"] in (128, 256, 512, 1024)
    for s in auto:
        ctx.tune(oc.OC_TUNE_SURF_BINS, s, 0)
    ctx.tune(oc.OC_TUNE_EXACT_WAVES, 0, 0)
    ctx.tune(oc.OC_TUNE_FILTER_BLOCK, 0, 0)
    with pytest.raises(oc.OcError):
        ctx.tune(99, 0, 0)
    with pytest.raises(oc.OcError):
        ctx.tune(oc.OC_TUNE_FILTER_BLOCK, 0, 96)
    # the tuning file: a new context applies it at creation
    path = str(tmp_path / "tune.txt")
    params["bin_factor"] = {str(autotune.size_class(n)): 0.5 for n in faces.values()}
    autotune.save(params, path)
    assert autotune.load(path) == params
    ctx2 = oc.Context(device=0, tune_cache=path)
    try:
        assert ctx2.tune(oc.OC_TUNE_EXACT_WAVES, 0, -1) == params["exact_waves"]
        assert ctx2.tune(oc.OC_TUNE_FILTER_BLOCK, 0, -1) == params["filter_block"]
        ids2 = _register(ctx2, cases)
        for (g, s), (g1, s1) in zip(ids2, ids):
            assert ctx2.tune(oc.OC_TUNE_SURF_BINS, s, -1) == max(1, int(auto[s1] * 0.5 + 0.5))
        outs2 = [torch.full((c["bg"].n_elem,), 5, dtype=torch.int8, device="cuda") for c in cases]
        ctx2.cut_batch([(g, [s], c["poses"][0].reshape(1, 12), ib) for (g, s), c, ib in zip(ids2, cases, outs2)])
        torch.cuda.synchronize()
        for a, b in zip(ref, outs2):
            assert np.array_equal(a, b.cpu().numpy())
    finally:
        torch.cuda.synchronize()
        ctx2.close()
    bad = tmp_path / "bad.txt"
    bad.write_text("filter_block 300\n")
    with pytest.raises(oc.OcError) as e:
        oc.Context(device=0, tune_cache=str(bad))
    assert e.value.status == oc.OC_EINVAL
