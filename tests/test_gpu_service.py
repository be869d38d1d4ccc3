"""The cut service (oc_submit / oc_wait): requests submitted back to back run
on slots of their own and each gives the iblank of the same request cut
alone and the oracle's; the HBM budget and the slot limit bound how many
run at once without changing any result; ticket and argument rules."""
import sys

import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def _cases(n):
    specs = CF.batch_instances(n=n, n_lo=8, n_hi=22, m_lo=3, m_hi=8)
    return [CF.batch_case(s, layers=2) for s in specs]


def _register(ctx, cases):
    return [(ctx.register_grid(c["bg"].nodes, c["bg"].conn),
             ctx.register_cut_surface(c["bodies"][0]["surface"].nodes, c["bodies"][0]["surface"].conn))
            for c in cases]


def _solo(ctx, gid, sids, poses, n_elem):
    import torch
    out = torch.empty(n_elem, dtype=torch.int8, device="cuda")
    ctx.cut_multi(gid, sids, poses, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_service_matches_solo_and_oracle(orc):
    import torch
    from paper_1711_07663_amd import oc
    _note("service: 8 uneven instances + union request, waited in reverse order")
    ctx = oc.Context(device=0)
    try:
        cases = _cases(8)
        ids = _register(ctx, cases)
        outs = []
        tickets = []
        for (g, s), c in zip(ids, cases):
            ib = torch.empty(c["bg"].n_elem, dtype=torch.int8, device="cuda")
            # written on the context stream before the submission: the
            # request is ordered after it
            with torch.cuda.stream(ctx.stream):
                ib.fill_(7)
            tickets.append(ctx.submit(g, [s], c["poses"][0].reshape(1, 12), ib))
            outs.append(ib)
        # a union of two surfaces and a request with no surface
        bg = M.background_grid(18, -1.5, 1.5, amp=0.02)
        s1 = M.cube_sphere(5, R=0.4, dimples=12, dimple_a=0.07, dimple_k=0.015)
        s2 = M.cube_sphere(4, R=0.3, axes=(0.3, 0.22, 0.18))
        g = ctx.register_grid(bg.nodes, bg.conn)
        a = ctx.register_cut_surface(s1.nodes, s1.conn)
        b = ctx.register_cut_surface(s2.nodes, s2.conn)
        pa, pb = M.pose_rz(0.3, (-0.45, 0.1, 0.0)), M.pose_rz(-0.7, (0.55, -0.05, 0.1))
        ib_u = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        ib_0 = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        t_u = ctx.submit(g, [a, b], np.stack([pa, pb]), ib_u)
        t_0 = ctx.submit(g, [], None, ib_0)
        info = ctx.service_info()
        assert 1 <= info["slots"] <= 4 and info["peak_running"] >= 1
        assert ctx.wait(t_0) and ctx.wait(t_u)
        for t in reversed(tickets):
            assert ctx.wait(t)
        for (gid, s), c, ib in zip(ids, cases, outs):
            got = ib.cpu().numpy()
            assert np.array_equal(got, _solo(ctx, gid, [s], c["poses"][0], c["bg"].n_elem)), c["name"]
            assert np.array_equal(got, orc.cut(c["bg"], [c["bodies"][0]["surface"]], c["poses"])), c["name"]
        assert np.array_equal(ib_u.cpu().numpy(), orc.cut(bg, [s1, s2], [pa, pb]))
        assert np.array_equal(ib_0.cpu().numpy(), orc.cut(bg, [], []))
        info = ctx.service_info()
        assert info["running"] == 0 and info["queued"] == 0 and info["finished"] == 0
        assert info["peak_running"] <= 4
    finally:
        torch.cuda.synchronize()
        ctx.close()


def _same_shape_requests():
    bg = M.background_grid(20, -1.5, 1.5, amp=0.03)
    s = M.cube_sphere(5, R=0.45, dimples=14, dimple_a=0.08, dimple_k=0.02)
    rng = np.random.default_rng(76)
    return bg, s, [M.random_pose(rng, 0.25) for _ in range(5)]


def _slot_and_base_bytes(bg, s, pose):
    """Device bytes of the registered state and of one service slot for a
    request of this shape, measured on an unbudgeted context."""
    import torch
    from paper_1711_07663_amd import oc
    ctx = oc.Context(device=0)
    try:
        g, sid = ctx.register_grid(bg.nodes, bg.conn), ctx.register_cut_surface(s.nodes, s.conn)
        base = ctx.memory_used()
        ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        assert ctx.wait(ctx.submit(g, [sid], pose.reshape(1, 12), ib))
        slot = ctx.service_info()["slot_bytes"]
        assert ctx.memory_used() == base + slot
        return base, slot, ib.cpu().numpy()
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_service_budget_admits_one_at_a_time(orc):
    """A budget with room for one slot: five requests queue behind each
    other, run one at a time and give the unbudgeted results."""
    import torch
    from paper_1711_07663_amd import oc
    _note("service: budget for one slot, 5 requests")
    bg, s, poses = _same_shape_requests()
    base, slot, first = _slot_and_base_bytes(bg, s, poses[0])
    ctx = oc.Context(device=0)
    try:
        g, sid = ctx.register_grid(bg.nodes, bg.conn), ctx.register_cut_surface(s.nodes, s.conn)
        assert ctx.memory_used() == base
        assert ctx.tune(oc.OC_TUNE_HBM_BUDGET, 0, base + slot + slot // 2) == base + slot + slot // 2
        outs = [torch.empty(bg.n_elem, dtype=torch.int8, device="cuda") for _ in poses]
        tickets = [ctx.submit(g, [sid], p.reshape(1, 12), ib) for p, ib in zip(poses, outs)]
        for t in tickets:
            assert ctx.wait(t)
        info = ctx.service_info()
        assert info["slots"] == 1 and info["peak_running"] == 1
        assert np.array_equal(outs[0].cpu().numpy(), first)
        for p, ib in zip(poses, outs):
            assert np.array_equal(ib.cpu().numpy(), orc.cut(bg, [s], [p]))
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_service_refuses_what_never_fits():
    import torch
    from paper_1711_07663_amd import oc
    _note("service: request larger than the budget")
    bg, s, poses = _same_shape_requests()
    base, slot, _ = _slot_and_base_bytes(bg, s, poses[0])
    ctx = oc.Context(device=0)
    try:
        g, sid = ctx.register_grid(bg.nodes, bg.conn), ctx.register_cut_surface(s.nodes, s.conn)
        ctx.tune(oc.OC_TUNE_HBM_BUDGET, 0, base + slot // 2)
        ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        with pytest.raises(oc.OcError) as e:
            ctx.submit(g, [sid], poses[0].reshape(1, 12), ib)
        assert e.value.status == oc.OC_EBUDGET
        info = ctx.service_info()
        assert info["slots"] == 0 and info["queued"] == 0 and info["running"] == 0
        assert ctx.memory_used() == base
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_service_slot_limit_and_reuse():
    """One slot allowed: requests of two shapes take turns, the slot is
    replaced when it does not cover the next request, results unchanged."""
    import torch
    from paper_1711_07663_amd import oc
    _note("service: slot limit 1, two request shapes")
    ctx = oc.Context(device=0)
    try:
        assert ctx.tune(oc.OC_TUNE_SERVICE_SLOTS, 0, 1) == 1
        cases = _cases(4)
        ids = _register(ctx, cases)
        outs = [torch.empty(c["bg"].n_elem, dtype=torch.int8, device="cuda") for c in cases]
        tickets = [ctx.submit(g, [s], c["poses"][0].reshape(1, 12), ib) for (g, s), c, ib in zip(ids, cases, outs)]
        for t in tickets:
            assert ctx.wait(t)
        info = ctx.service_info()
        assert info["slots"] == 1 and info["peak_running"] == 1
        for (g, s), c, ib in zip(ids, cases, outs):
            assert np.array_equal(ib.cpu().numpy(), _solo(ctx, g, [s], c["poses"][0], c["bg"].n_elem))
        assert ctx.tune(oc.OC_TUNE_SERVICE_SLOTS, 0, 0) == 4
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_service_ticket_and_argument_rules():
    import torch
    from paper_1711_07663_amd import oc
    _note("service: tickets, timeouts, invalid requests")
    ctx = oc.Context(device=0)
    try:
        bg, s, poses = _same_shape_requests()
        g, sid = ctx.register_grid(bg.nodes, bg.conn), ctx.register_cut_surface(s.nodes, s.conn)
        with pytest.raises(oc.OcError) as e:
            ctx.wait(12345)
        assert e.value.status == oc.OC_ENOTFOUND
        ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        t = ctx.submit(g, [sid], poses[0].reshape(1, 12), ib)
        # the same output again before the first request was waited for
        with pytest.raises(oc.OcError) as e:
            ctx.submit(g, [sid], poses[1].reshape(1, 12), ib)
        assert e.value.status == oc.OC_EINVAL
        polled = ctx.wait(t, timeout_ms=0)
        assert polled in (True, False)
        if not polled:
            assert ctx.wait(t)
        with pytest.raises(oc.OcError) as e:
            ctx.wait(t)
        assert e.value.status == oc.OC_ENOTFOUND
        # reusable once waited for
        assert ctx.wait(ctx.submit(g, [sid], poses[1].reshape(1, 12), ib))
        with pytest.raises(oc.OcError) as e:
            ctx.submit(g, [sid + 10], poses[0].reshape(1, 12), ib)
        assert e.value.status == oc.OC_ENOTFOUND
        bad = poses[0].copy()
        bad[3] = np.nan
        with pytest.raises(oc.OcError) as e:
            ctx.submit(g, [sid], bad.reshape(1, 12), ib)
        assert e.value.status == oc.OC_EINVAL
        wide = torch.empty(bg.n_elem + 4, dtype=torch.int8, device="cuda")
        with pytest.raises(oc.OcError) as e:   # not 4-byte aligned
            ctx.submit(g, [sid], poses[0].reshape(1, 12), wide[1:1 + bg.n_elem])
        assert e.value.status == oc.OC_EINVAL
        # a queued request is dropped with the context
        ib2 = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
        ctx.submit(g, [sid], poses[2].reshape(1, 12), ib2)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_service_cancel_queued_request():
    """With one service slot held by a request that waits behind work on the
    context stream, a second request stays queued: cancelling it forgets its
    ticket and leaves its output untouched; the running one cannot be
    cancelled and finishes with the solo result; later requests run."""
    import torch
    from paper_1711_07663_amd import oc
    _note("service: cancel a queued request")
    ctx = oc.Context(device=0)
    try:
        assert ctx.tune(oc.OC_TUNE_SERVICE_SLOTS, 0, 1) == 1
        bg, s, poses = _same_shape_requests()
        g, sid = ctx.register_grid(bg.nodes, bg.conn), ctx.register_cut_surface(s.nodes, s.conn)
        outs = [torch.full((bg.n_elem,), 7, dtype=torch.int8, device="cuda") for _ in range(3)]
        torch.cuda.synchronize()
        with torch.cuda.stream(ctx.stream):
            torch.cuda._sleep(200_000_000)       # about 0.1 s of spinning on the context stream
        ta = ctx.submit(g, [sid], poses[0].reshape(1, 12), outs[0])
        tb = ctx.submit(g, [sid], poses[1].reshape(1, 12), outs[1])
        info = ctx.service_info()
        assert info["running"] == 1 and info["queued"] == 1
        assert ctx.cancel(tb) is True
        assert ctx.service_info()["queued"] == 0
        assert ctx.cancel(ta) is False
        with pytest.raises(oc.OcError) as e:
            ctx.cancel(987654)
        assert e.value.status == oc.OC_ENOTFOUND
        assert ctx.wait(ta)
        with pytest.raises(oc.OcError) as e:
            ctx.wait(tb)
        assert e.value.status == oc.OC_ENOTFOUND
        torch.cuda.synchronize()
        assert (outs[1].cpu().numpy() == 7).all()
        assert np.array_equal(outs[0].cpu().numpy(), _solo(ctx, g, [sid], poses[0], bg.n_elem))
        tc = ctx.submit(g, [sid], poses[2].reshape(1, 12), outs[2])
        assert ctx.wait(tc)
        with pytest.raises(oc.OcError) as e:     # forgotten once waited for
            ctx.cancel(tc)
        assert e.value.status == oc.OC_ENOTFOUND
        assert np.array_equal(outs[2].cpu().numpy(), _solo(ctx, g, [sid], poses[2], bg.n_elem))
    finally:
        torch.cuda.synchronize()
        ctx.close()
