"""The allocation-free donor search (oc_donor_search_noalloc) against the
allocating one (oc_donor_search), through the C ABI, on two calls in a row
(the second smaller, at another pose), on a shell grid and on a curved
background.  Bar: donor ids equal, reference coordinates within 1e-10, NaN
for the same orphans; the context holds no more device memory after the
calls than before."""
import sys

import numpy as np
import pytest

from workloads import meshes as M

pytestmark = pytest.mark.gpu

XI_TOL = 1e-10


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1711_07663_amd import oc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = oc.Context(device=0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _points(rng, n, lo, hi):
    return rng.uniform(lo, hi, size=(n, 3))


def _search_both(ctx, gid, pose, pts_host):
    import torch
    n = pts_host.shape[0]
    pts = torch.from_numpy(np.ascontiguousarray(pts_host)).cuda()
    d_a = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    r_a = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    d_b = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    r_b = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    used0 = ctx.memory_used()
    torch_used0 = torch.cuda.memory_allocated()
    ctx.donor_search_noalloc(gid, pose, pts, n, d_a, r_a)
    torch.cuda.synchronize()
    assert ctx.memory_used() == used0, "the allocation-free search changed the context's device memory"
    assert torch.cuda.memory_allocated() == torch_used0
    ctx.donor_search(gid, pose, pts, n, d_b, r_b)
    torch.cuda.synchronize()
    return d_a.cpu().numpy(), r_a.cpu().numpy(), d_b.cpu().numpy(), r_b.cpu().numpy()


def _check_equal(d_a, r_a, d_b, r_b, what):
    bad = np.nonzero(d_a != d_b)[0]
    assert bad.size == 0, "%s: %d donor ids differ, first %s: noalloc %s alloc %s" % (
        what, bad.size, bad[:5], d_a[bad[:5]], d_b[bad[:5]])
    ok = d_b >= 0
    assert ok.any() and (~ok).any(), what + ": the case should hold donors and orphans"
    err = np.abs(r_a[ok] - r_b[ok]).max()
    assert err <= XI_TOL, "%s: max |xi_noalloc - xi_alloc| = %g" % (what, err)
    assert np.all(np.isnan(r_a[~ok])), what + ": orphans must get NaN reference coordinates"


def test_noalloc_matches_donor_search_two_calls(ctx):
    from paper_1711_07663_amd import oc
    rng = np.random.default_rng(4242)
    nmax = oc.Context.noalloc_max_points()
    assert nmax >= 1 << 16
    # a curved background (the sinusoidal displacement) and a posed shell
    bg = M.background_grid(24, -1.5, 1.5, amp=0.03)
    s = M.cube_sphere(8, R=0.5, dimples=20, dimple_a=0.09, dimple_k=0.025)
    sh = M.shell_grid(s, 4, r_out=1.0)
    g_bg = ctx.register_grid(bg.nodes, bg.conn)
    g_sh = ctx.register_grid(sh.nodes, sh.conn, sh.face_tags)

    _note("noalloc call 1: background, %d points (limit %d)" % (nmax, nmax))
    pts = _points(rng, nmax, -1.6, 1.6)     # some outside the grid: orphans
    _check_equal(*_search_both(ctx, g_bg, M.IDENTITY_POSE, pts), "background, full-size call")

    pose = M.random_pose(rng, 0.2)
    _note("noalloc call 2: posed shell, 9000 points")
    pts2 = M.apply_pose_to_points(pose, _points(rng, 9000, -1.05, 1.05))
    _check_equal(*_search_both(ctx, g_sh, pose, pts2), "posed shell, smaller call")

    _note("noalloc call 3: background again, 1234 points")
    pts3 = _points(rng, 1234, -1.6, 1.6)
    _check_equal(*_search_both(ctx, g_bg, M.IDENTITY_POSE, pts3), "background, small call after a small call")


def test_noalloc_limits(ctx):
    import torch
    from paper_1711_07663_amd import oc
    bg = M.background_grid(6, -1.0, 1.0, amp=0.0)
    gid = ctx.register_grid(bg.nodes, bg.conn)
    nmax = oc.Context.noalloc_max_points()
    _note("noalloc limits: n = 0 and n = %d + 1" % nmax)
    ctx.donor_search_noalloc(gid, M.IDENTITY_POSE, None, 0, None, None)   # nothing to do
    big = torch.zeros((nmax + 1, 3), dtype=torch.float64, device="cuda")
    d = torch.zeros(nmax + 1, dtype=torch.int32, device="cuda")
    r = torch.zeros((nmax + 1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(oc.OcError) as e:
        ctx.donor_search_noalloc(gid, M.IDENTITY_POSE, big, nmax + 1, d, r)
    assert e.value.status == oc.OC_EINVAL
    with pytest.raises(oc.OcError) as e:
        ctx.donor_search_noalloc(gid + 1000, M.IDENTITY_POSE, big, 10, d, r)
    assert e.value.status in (oc.OC_EINVAL, oc.OC_ENOTFOUND)
    # the device is still usable after the refusals
    pts = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    ctx.donor_search_noalloc(gid, M.IDENTITY_POSE, pts, 4, d, r)
    torch.cuda.synchronize()
    assert (d[:4].cpu().numpy() >= 0).all()
