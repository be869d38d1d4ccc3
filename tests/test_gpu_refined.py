"""The HIP refined cut (oc_cut_refined: surface faces split k x k, near
elements k^3 times, an element a hole when one of its sub-elements is)
against the oracle's refined cut on the same seeded inputs.  Bar: iblank
bit-exact.  Level 1 must equal the lattice cut (oc_cut_multi); the cases
are chosen so that levels 2 and 3 change the status of some elements
(checked on the oracle side), so equality is not reached by the lattice cut
alone."""
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
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = oc.Context(device=0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _case(name):
    if name == "tiny":
        case = CF.tiny()
        return case["bg"], [case["bodies"][0]["surface"]], [M.IDENTITY_POSE]
    if name == "dimpled12":
        rng = np.random.default_rng(7)
        bg = M.background_grid(12, -1.0, 1.0, amp=0.05)
        s = M.cube_sphere(4, R=0.5, dimples=12, dimple_a=0.1, dimple_k=0.03)
        return bg, [s], [M.random_pose(rng, 0.1)]
    if name == "coarse-sphere20":
        rng = np.random.default_rng(7)
        M.random_pose(rng, 0.1)
        bg = M.background_grid(20, -1.0, 1.0, amp=0.04)
        s = M.cube_sphere(3, R=0.45)
        return bg, [s], [M.random_pose(rng, 0.1)]
    if name == "two-bodies":
        rng = np.random.default_rng(21)
        bg = M.background_grid(16, -1.2, 1.2, amp=0.05)
        a = M.cube_sphere(3, R=0.35, dimples=8, dimple_a=0.08, dimple_k=0.03)
        b = M.cube_sphere(3, R=0.3)
        pa = M.random_pose(rng, 0.05)
        pa[9:12] += np.array([-0.4, 0.05, 0.0])
        pb = M.random_pose(rng, 0.05)
        pb[9:12] += np.array([0.45, -0.1, 0.1])
        return bg, [a, b], [pa, pb]
    if name == "dimpled40":
        rng = np.random.default_rng(11)
        bg = M.background_grid(40, -1.5, 1.5, amp=0.04)
        s = M.cube_sphere(8, R=0.6, dimples=50, dimple_a=0.08, dimple_k=0.03)
        return bg, [s], [M.random_pose(rng, 0.1)]
    raise KeyError(name)


def _run(ctx, bg, surfs, poses, k):
    import torch
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sids = [ctx.register_cut_surface(s.nodes, s.conn) for s in surfs]
    ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    n_near = ctx.cut_refined(gid, sids, np.stack(poses), ib, k)
    return gid, sids, ib, n_near


def _compare(got, want, what):
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s: %d elements differ, first %s: gpu %s oracle %s" % (
        what, bad.size, bad[:8], got[bad[:8]], want[bad[:8]])


CASES = [("tiny", 2), ("tiny", 3), ("dimpled12", 2), ("dimpled12", 3), ("coarse-sphere20", 2),
         ("coarse-sphere20", 4), ("two-bodies", 2), ("dimpled40", 2)]


@pytest.mark.parametrize("name,k", CASES)
def test_refined_cut_parity(ctx, orc, name, k):
    _note("refined cut %s level %d" % (name, k))
    bg, surfs, poses = _case(name)
    _, _, ib, n_near = _run(ctx, bg, surfs, poses, k)
    want = orc.cut_refined(bg, surfs, poses, k)
    _compare(ib.cpu().numpy(), want, "%s level %d" % (name, k))
    assert n_near > 0
    if name != "tiny":
        lattice = orc.cut(bg, surfs, poses)
        assert (lattice != want).any(), "the case must separate level %d from the lattice cut" % k


@pytest.mark.parametrize("name", ["tiny", "dimpled12", "two-bodies"])
def test_level_one_is_the_lattice_cut(ctx, name):
    import torch
    _note("refined cut %s level 1 against oc_cut_multi" % name)
    bg, surfs, poses = _case(name)
    gid, sids, ib, _ = _run(ctx, bg, surfs, poses, 1)
    ref = torch.empty_like(ib)
    ctx.cut_multi(gid, sids, np.stack(poses), ref)
    assert torch.equal(ib, ref)


def test_flat_faces_on_a_box_grid(ctx, orc):
    _note("refined cut of a box surface on an undisplaced grid")
    g = M.background_grid(10, -1.5, 1.5, amp=0.0)
    s = M.box_surface(2, (-0.41, 0.63, -0.2), (0.37, 0.88, 0.61))
    _, _, ib3, _ = _run(ctx, g, [s], [M.IDENTITY_POSE], 3)
    _compare(ib3.cpu().numpy(), orc.cut(g, [s], [M.IDENTITY_POSE]), "box level 3")


def test_bad_arguments(ctx):
    import torch
    from paper_1711_07663_amd import oc
    _note("refined cut argument checks")
    bg, surfs, poses = _case("dimpled12")
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(surfs[0].nodes, surfs[0].conn)
    ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    for k in (0, 9):
        with pytest.raises(oc.OcError):
            ctx.cut_refined(gid, [sid], np.stack(poses), ib, k)
    bad = np.array(poses[0], dtype=np.float64)
    bad[10] = np.nan
    with pytest.raises(oc.OcError):
        ctx.cut_refined(gid, [sid], bad[None], ib, 2)


def test_full_size_sampled(ctx, orc):
    """The dimpled 128^3 case at level 2: every element whose blanking
    differs from the lattice cut, and random band elements and holes, one by
    one against the oracle's definition (hole when one of the element's
    sub-elements is a hole of the refined surface); holes only inside the
    band; the fringe layer of the HIP hole mask."""
    import torch
    _note("refined cut of the dimpled 128^3 case, level 2, sampled")
    case = CF.dimpled()
    bg, s = case["bg"], case["bodies"][0]["surface"]
    pose = np.asarray(case["poses"][0], dtype=np.float64)
    k = 2
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    lat_t = torch.empty_like(ib)
    ctx.cut_refined(gid, [sid], pose[None], ib, k)
    ctx.cut(gid, sid, pose, lat_t)
    got, lat = ib.cpu().numpy(), lat_t.cpu().numpy()
    hole = got == orc.HOLE
    # band of the oracle's refined cut: control-net boxes within 1e-4 of the
    # posed refined surface's box
    sv = orc.refine_surface(s, k)
    R = pose[:9].reshape(3, 3)
    Y = sv.nodes @ R.T + pose[9:12]
    slo, shi = Y.min(axis=0) - 1e-4, Y.max(axis=0) + 1e-4
    band = []
    for s0 in range(0, bg.n_elem, 1 << 16):
        ids = np.arange(s0, min(bg.n_elem, s0 + (1 << 16)))
        lo, hi = orc._control_boxes(bg, ids)
        band.append(ids[np.all(hi >= slo, axis=1) & np.all(lo <= shi, axis=1)])
    band = np.concatenate(band)
    in_band = np.zeros(bg.n_elem, dtype=bool)
    in_band[band] = True
    assert not (hole & ~in_band).any()
    changed = np.nonzero((got == orc.HOLE) != (lat == orc.HOLE))[0]
    assert changed.size > 0, "curvature must change some elements at this size"
    rng = np.random.default_rng(1711)
    holes = np.nonzero(hole)[0]
    sample = np.unique(np.concatenate([changed, rng.choice(band, 150, replace=False),
                                       rng.choice(holes, 50, replace=False)]))
    sub = orc.refine_elements(bg, sample, k)
    st = orc.cut_surface(sub, sv, pose)
    want = (st.reshape(sample.size, k ** 3) == 0).any(axis=1)
    bad = sample[want != hole[sample]]
    assert bad.size == 0, "%d sampled elements differ, first %s" % (bad.size, bad[:8])
    nbr = orc.face_neighbors(bg.conn)
    assert np.array_equal(orc.mark_fringe(hole, nbr, bg.face_tags), got)
