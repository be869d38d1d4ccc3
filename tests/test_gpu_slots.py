"""Slots (pre-reserved per-request scratch, device poses and counts) and
graph replay against the default path and the oracle."""
import sys

import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M

from parity_util import compare, oracle_step

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


def _small_case():
    bg = M.background_grid(20, -1.4, 1.4, amp=0.03)
    s = M.cube_sphere(6, R=0.5, dimples=30, dimple_a=0.08, dimple_k=0.02)
    sh = M.shell_grid(s, 3, r_out=0.95)
    return dict(bg=bg, bodies=[dict(surface=s, shell=sh)])


def _snapshot(system, counts):
    n_bg = counts["n_bg_points"]
    out = dict(ib_bg=system.ib_bg.cpu().numpy(), pts_bg=system.pts_bg[:n_bg].cpu().numpy(),
               src_bg=system.src_bg[:n_bg].cpu().numpy(), bodies=[])
    for b, n in zip(system.bodies, counts["n_shell_points"]):
        out["bodies"].append(dict(ib=b["ib"].cpu().numpy(), pts=b["pts"][:n].cpu().numpy(),
                                  src=b["src"][:n].cpu().numpy(), donor_bg=b["donor_bg"][:n_bg].cpu().numpy(),
                                  ref_bg=b["ref_bg"][:n_bg].cpu().numpy(), donor=b["donor"][:n].cpu().numpy(),
                                  ref=b["ref"][:n].cpu().numpy()))
    return out


def _equal(a, b):
    assert np.array_equal(a["ib_bg"], b["ib_bg"])
    assert np.array_equal(a["pts_bg"], b["pts_bg"])
    for x, y in zip(a["bodies"], b["bodies"]):
        for k in ("ib", "pts", "src", "donor_bg", "donor"):
            assert np.array_equal(x[k], y[k]), k
        for k in ("ref_bg", "ref"):
            assert np.array_equal(x[k], y[k], equal_nan=True), k


def test_slot_step_matches_oracle_and_default_path(ctx, orc):
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("slot eager step vs default path vs oracle (small dimpled case)")
    case = _small_case()
    system = OversetSystem(ctx, case)
    rng = np.random.default_rng(7)
    poses = [M.random_pose(rng, 0.15)]
    c0 = system.step(poses)
    torch.cuda.synchronize()
    ref = _snapshot(system, c0)
    ss = SlotStep(system)
    ss.step(poses)
    got = ss.snapshot()
    _equal(ref, got)
    compare(got, oracle_step(case, poses))


def test_graph_replay_matches_eager(ctx, orc):
    """Replays interleaved with eager work and synchronisations; every replay
    equals the eager step for the same poses."""
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("graph replay of a moving body, 6 poses, interleaved with eager steps")
    case = _small_case()
    system = OversetSystem(ctx, case)
    ss = SlotStep(system)
    poses = [[M.pose_rz(0.05 * k, (0.01 * k, 0.0, -0.005 * k))] for k in range(6)]
    ss.step(poses[0])
    torch.cuda.synchronize()
    ss.capture()
    for k, p in enumerate(poses):
        ss.step(p)
        eager = ss.snapshot()
        ss.replay(poses[(k + 3) % len(poses)])
        torch.cuda.synchronize()
        ss.replay(p)
        _equal(eager, ss.snapshot())
    compare(ss.snapshot(), oracle_step(case, poses[-1]))


def test_two_slots_concurrent(ctx):
    """Two SlotSteps of one system on two streams, launched back to back
    without synchronisation, give the results each gives alone."""
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("two slots of one system on two streams concurrently")
    case = _small_case()
    system = OversetSystem(ctx, case)
    ta, tb = SlotStep(system), SlotStep(system)
    pa, pb = [M.pose_rz(0.3, (0.05, 0, 0))], [M.pose_rz(-0.2, (0, 0.04, 0.02))]
    ta.step(pa)
    solo_a = ta.snapshot()
    tb.step(pb)
    solo_b = tb.snapshot()
    for _ in range(3):
        ta.step(pa)
        tb.step(pb)
        torch.cuda.synchronize()
        _equal(solo_a, ta.snapshot())
        _equal(solo_b, tb.snapshot())


def test_warm_slot_graph_spinning(ctx, orc):
    """The spinning-body step: cold first step, then warm-started graph
    replays (two parities) over 8 poses; each equals a cold eager step at
    the same pose, and the last equals the oracle."""
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("warm-started graph replay of a spinning dimpled sphere, 8 steps")
    case = _small_case()
    system = OversetSystem(ctx, case)
    poses = [[M.pose_rz(2 * np.pi * k / 50)] for k in range(9)]
    sweep = ctx.sweep_bound(system.bodies[0]["surf"], poses[0][0], poses[1][0])
    warm = SlotStep(system, warm=True, sweep=sweep)
    cold = SlotStep(system)
    warm.step(poses[0])
    torch.cuda.synchronize()
    warm.capture()
    for k in range(1, len(poses)):
        warm.replay(poses[k])
        got = warm.snapshot()
        cold.step(poses[k])
        _equal(cold.snapshot(), got)
    compare(got, oracle_step(case, poses[-1]))


def test_warm_slot_pose_jump_runs_cold(ctx, orc):
    """A warm step whose pose moved farther than the sweep bound the step was
    built with runs cold (eagerly) instead of keeping stale statuses; steps
    within the bound stay on the warm graph."""
    import torch
    from paper_1711_07663_amd.pipeline import OversetSystem, SlotStep
    _note("warm-started step with a pose jump beyond its sweep bound")
    case = _small_case()
    system = OversetSystem(ctx, case)
    step = 2 * np.pi / 50
    sweep = ctx.sweep_bound(system.bodies[0]["surf"], M.pose_rz(0.0), M.pose_rz(step))
    warm = SlotStep(system, warm=True, sweep=sweep)
    cold = SlotStep(system)
    warm.step([M.pose_rz(0.0)])
    torch.cuda.synchronize()
    warm.capture()
    seq = [step, 2 * step, 2 * step + 0.9, 3 * step + 0.9, 0.1]   # jumps at the third and fifth
    for k, th in enumerate(seq):
        warm.replay([M.pose_rz(th)])
        got = warm.snapshot()
        cold.step([M.pose_rz(th)])
        _equal(cold.snapshot(), got)
    assert warm.cold_fallbacks == 2
    compare(got, oracle_step(case, [M.pose_rz(seq[-1])]))


def test_slot_budget(ctx):
    from paper_1711_07663_amd import oc
    _note("slot creation over the HBM budget")
    small = oc.Context(device=0, hbm_budget=64 << 20)
    g = M.background_grid(24, -1, 1)
    gid = small.register_grid(g.nodes, g.conn)
    used = small.memory_used()
    assert used < (64 << 20)
    slots = []
    with pytest.raises(oc.OcError) as ei:
        for _ in range(1000):
            slots.append(small.create_slot([gid], []))
    assert ei.value.status == oc.OC_EBUDGET
    assert len(slots) >= 1
    for sl in slots:
        sl.close()
    assert small.memory_used() == used
    small.close()


def test_warm_start_equals_cold(ctx, orc):
    """Spinning body: every warm-started cut equals the cold cut at the same
    pose (and the oracle at a few poses)."""
    import torch
    _note("warm start over 12 poses of a spinning dimpled sphere")
    bg = M.background_grid(24, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(8, R=0.5, dimples=40, dimple_a=0.07, dimple_k=0.02)
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    poses = [M.pose_rz(2 * np.pi * k / 40, (0.0, 0.0, 0.01 * k)) for k in range(12)]
    prev = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    cur = torch.empty_like(prev)
    cold = torch.empty_like(prev)
    ctx.cut(gid, sid, poses[0], prev)
    for k in range(1, len(poses)):
        ctx.cut_warm(gid, sid, poses[k], poses[k - 1], prev, cur)
        ctx.cut(gid, sid, poses[k], cold)
        torch.cuda.synchronize()
        assert torch.equal(cur, cold), "step %d" % k
        if k in (1, 6, 11):
            assert np.array_equal(cur.cpu().numpy(), orc.cut(bg, [s], [poses[k]]))
        prev, cur = cur, prev
    assert ctx.sweep_bound(sid, poses[0], poses[1]) >= 0.5 * 2 * np.pi / 40


def test_slot_outlives_context():
    """Closing a context destroys its slots; a Slot object that outlives it
    becomes a closed handle (its calls fail cleanly, closing it is a no-op)."""
    import torch
    from paper_1711_07663_amd import oc
    _note("slot object outliving its context")
    c = oc.Context(device=0)
    g = M.background_grid(4, -1, 1)
    gid = c.register_grid(g.nodes, g.conn)
    sl = c.create_slot([gid], [])
    c.close()
    ib = torch.empty(g.n_elem, dtype=torch.int8, device="cuda")
    c.grids[gid] = g.n_elem
    with pytest.raises(oc.OcError):
        sl.cut(gid, [], None, ib)
    sl.close()
    del sl
