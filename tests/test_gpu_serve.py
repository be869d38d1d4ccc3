"""Serving with continuous batching: every request's outputs are the same
whether it runs alone or mixed with others in flight, under a budget that
admits many slots and under one that admits a single slot."""
import sys

import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def _systems(ctx):
    from paper_1711_07663_amd.pipeline import OversetSystem
    tiny = CF.tiny()
    bg = M.background_grid(20, -1.4, 1.4, amp=0.03)
    s = M.cube_sphere(6, R=0.5, dimples=30, dimple_a=0.08, dimple_k=0.02)
    small = dict(bg=bg, bodies=[dict(surface=s, shell=M.shell_grid(s, 3, r_out=0.95))])
    two = CF.two_body(bg_n=24, m=4, layers=2, dimples=0)
    return dict(tiny=OversetSystem(ctx, tiny), small=OversetSystem(ctx, small), two=OversetSystem(ctx, two))


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        k = ("tiny", "small", "two")[i % 3]
        if k == "two":
            out.append((k, CF.two_body_poses(int(rng.integers(0, 400)))))
        else:
            out.append((k, [M.random_pose(rng, 0.15)]))
    return out


def _solo(systems, reqs):
    import torch
    res = []
    for name, poses in reqs:
        sysm = systems[name]
        c = sysm.step(poses)
        torch.cuda.synchronize()
        n_bg = c["n_bg_points"]
        r = dict(ib_bg=sysm.ib_bg.cpu().numpy(), donor=[], ib=[])
        for b, n in zip(sysm.bodies, c["n_shell_points"]):
            r["ib"].append(b["ib"].cpu().numpy())
            r["donor"].append((b["donor_bg"][:n_bg].cpu().numpy(), b["ref_bg"][:n_bg].cpu().numpy(),
                               b["donor"][:n].cpu().numpy(), b["ref"][:n].cpu().numpy()))
        res.append(r)
    return res


def _served(ctx, systems, reqs, budget, max_slots):
    from paper_1711_07663_amd.serve import Server
    got = {}

    def on_done(req, ss):
        snap = ss.snapshot()
        got[req["tag"]] = dict(ib_bg=snap["ib_bg"], ib=[b["ib"] for b in snap["bodies"]],
                               donor=[(b["donor_bg"], b["ref_bg"], b["donor"], b["ref"]) for b in snap["bodies"]])

    srv = Server(ctx, systems, budget, max_slots=max_slots, on_done=on_done)
    # a burst (everything queued at once), then requests trickling in while
    # others are in flight
    half = len(reqs) // 2
    for i in range(half):
        srv.submit(reqs[i][0], reqs[i][1], tag=i)
    srv.pump()
    for i in range(half, len(reqs)):
        srv.submit(reqs[i][0], reqs[i][1], tag=i)
        srv.pump()
    srv.drain()
    return got, srv


def _same(a, b):
    assert np.array_equal(a["ib_bg"], b["ib_bg"])
    for x, y in zip(a["ib"], b["ib"]):
        assert np.array_equal(x, y)
    for x, y in zip(a["donor"], b["donor"]):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[2], y[2])
        assert np.array_equal(x[1], y[1], equal_nan=True) and np.array_equal(x[3], y[3], equal_nan=True)


def test_served_equals_solo():
    import torch
    from paper_1711_07663_amd import oc
    _note("serving: 24 mixed requests, many slots, vs solo")
    ctx = oc.Context(device=0)
    try:
        systems = _systems(ctx)
        reqs = _requests(24, 5)
        solo = _solo(systems, reqs)
        got, srv = _served(ctx, systems, reqs, budget=8 << 30, max_slots=8)
        assert len(got) == len(reqs)
        assert len(srv.slots) >= 3
        for i, r in enumerate(solo):
            _same(r, got[i])
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_served_tight_budget():
    import torch
    from paper_1711_07663_amd import oc
    from paper_1711_07663_amd.serve import Server
    _note("serving: budget for one slot")
    ctx = oc.Context(device=0)
    try:
        systems = _systems(ctx)
        reqs = _requests(9, 9)
        solo = _solo(systems, reqs)
        base = ctx.memory_used()
        probe = Server(ctx, systems, 1 << 40)
        need = max(probe.slot_size.values())
        got, srv = _served(ctx, systems, reqs, budget=base + need, max_slots=8)
        assert len(got) == len(reqs)
        assert srv.n_refused > 0
        for i, r in enumerate(solo):
            _same(r, got[i])
    finally:
        torch.cuda.synchronize()
        ctx.close()
