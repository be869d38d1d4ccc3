"""Input margins of the benchmark workloads (the inputs' geometric margin
from the cut surfaces, on which bit-exact parity rests), measured with the
oracle's exact element-surface distance, and a pin of the band method the
full-size parity tests use.

An element decides "intersected" by d < 1e-7 (d: its smallest triangle-pair
distance to the surface).  Both the oracle and the HIP path compute d in
FP64, with errors of order 1e-16 at these magnitudes; they agree when d is
exactly 0 (shared exact coordinates) or far from 1e-7.  Every element near
a surface is checked: d = 0, or d >= 1e-6, or, for the near-contacts listed
here (found by this measurement, a property of the generated inputs), d at
least 2e-7 away from 1e-7:

* dimpled 128^3 / spinning: none (smallest positive d 1.17e-6);
* 64-instance batch: instance 1 (46^3, sphere of 27^2 x 6 faces), one
  element at d = 3.18e-7;
* two-body: each shell's outer boundary touches the other sphere where the
  two meet on the x axis; at steps 0, 100 and 300 the contact is exact
  (d = 0: 4 elements, holes by the 1e-7 rule), and at steps 1, 2 and 399
  it is a near-contact (d = 3.3e-7 and 6.9e-7)."""
import numpy as np
import pytest

import parity_util as PU
from workloads import configs as CF
from workloads import meshes as M

TOL_HIT = 1e-7


def _near(orc, grid, surf, pose, pad=2e-6, boxes=None):
    """Exact distance of every element whose node box comes within pad of
    the node box of some posed surface face (every other element is farther
    than pad from the surface, whose triangles lie in their faces' boxes)."""
    from scipy.spatial import cKDTree
    R = np.asarray(pose[:9]).reshape(3, 3)
    X = (surf.nodes @ R.T + np.asarray(pose[9:12]))[surf.conn]
    flo, fhi = X.min(axis=1), X.max(axis=1)
    slo, shi = flo.min(axis=0) - pad, fhi.max(axis=0) + pad
    if boxes is None and grid.shape:
        # a generated background lattice: element (i, j, k) lies within its
        # undisplaced cell grown by the displacement amplitude (0.02 at most)
        n = np.asarray(grid.shape)
        glo, ghi = grid.nodes.min(axis=0), grid.nodes.max(axis=0)
        h = (ghi - glo) / n
        i0 = np.clip(np.floor((slo - 0.05 - glo) / h).astype(int) - 1, 0, n - 1)
        i1 = np.clip(np.floor((shi + 0.05 - glo) / h).astype(int) + 1, 0, n - 1)
        I, J, K = np.meshgrid(*[np.arange(i0[d], i1[d] + 1) for d in range(3)], indexing="ij")
        sub = (I + n[0] * (J + n[1] * K)).ravel()
        sg = type(grid)(nodes=grid.nodes, conn=grid.conn[sub])
        lo, hi = PU.element_boxes(sg)
        sel = sub[np.all(hi >= slo, axis=1) & np.all(lo <= shi, axis=1)]
        lo, hi = PU.element_boxes(type(grid)(nodes=grid.nodes, conn=grid.conn[sel]))
        lo_full = hi_full = None
    else:
        lo_full, hi_full = boxes if boxes is not None else PU.element_boxes(grid)
        sel = np.nonzero(np.all(hi_full >= slo, axis=1) & np.all(lo_full <= shi, axis=1))[0]
        lo, hi = lo_full[sel], hi_full[sel]
    # candidates by centre distance, then the exact box test
    if sel.size == 0:
        return sel, np.zeros(0)
    ec, er = 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo, axis=1)
    fc, fr = 0.5 * (flo + fhi), 0.5 * np.linalg.norm(fhi - flo, axis=1)
    cand = cKDTree(fc).query_ball_point(ec, er + fr.max() + pad)
    cnt = np.fromiter((len(c) for c in cand), dtype=np.int64, count=len(cand))
    ei = np.repeat(np.arange(sel.size), cnt)
    fi = np.fromiter((f for c in cand for f in c), dtype=np.int64, count=int(cnt.sum()))
    ok = np.all(fhi[fi] >= lo[ei] - pad, axis=1) & np.all(flo[fi] <= hi[ei] + pad, axis=1)
    band = sel[np.bincount(ei[ok], minlength=sel.size) > 0]
    if band.size == 0:
        return band, np.zeros(0)
    d = orc.cut_surface(grid, surf, pose, sel=band, diagnostics=True)["dstar"]
    return band, d


def _contacts(band, d):
    """(exact contacts, near-contacts as {element: d}) and the check that
    every element is decided far from the threshold."""
    near = (d > 0) & (d < 1e-6)
    assert np.all(np.abs(d[near] - TOL_HIT) >= 2e-7), "an element within 2e-7 of the hit threshold"
    return int((d == 0).sum()), {int(e): float(v) for e, v in zip(band[near], d[near])}


def test_band_method_equals_whole_grid(orc):
    """The band method gives the oracle's whole-grid iblank (tiny case; a
    posed two-body case whose shells are cut by the other wall)."""
    case = CF.tiny()
    assert np.array_equal(PU.band_cut(case["bg"], [case["bodies"][0]["surface"]], case["poses"]),
                          orc.cut(case["bg"], [case["bodies"][0]["surface"]], case["poses"]))
    two = CF.two_body(bg_n=20, m=6, layers=3, dimples=20)
    poses = CF.two_body_poses(3)
    walls = [b["surface"] for b in two["bodies"]]
    assert np.array_equal(PU.band_cut(two["bg"], walls, poses), orc.cut(two["bg"], walls, poses))
    rel = PU.pose_compose(PU.pose_inverse(poses[0]), poses[1])
    sh = two["bodies"][0]["shell"]
    assert np.array_equal(PU.band_cut(sh, [walls[1]], [rel]), orc.cut(sh, [walls[1]], [rel]))


def test_margin_tiny(orc):
    case = CF.tiny()
    d = orc.cut_surface(case["bg"], case["bodies"][0]["surface"], diagnostics=True)["dstar"]
    n0, near = _contacts(np.arange(d.size), d)
    assert near == {}
    assert n0 == 80          # 56 crossing + 24 exact contacts at the face-centre vertices on the axes


@pytest.mark.slow
def test_margin_dimpled_and_spinning(orc):
    case = CF.dimpled()
    bg, s = case["bg"], case["bodies"][0]["surface"]
    for pose in [M.IDENTITY_POSE] + [CF.spinning_poses(n)[-1] for n in (1, 100, 200)]:
        band, d = _near(orc, bg, s, pose)
        _, near = _contacts(band, d)
        assert near == {}
        assert d.size > 2000 and d[d > 0].min() >= 1e-6


@pytest.mark.slow
def test_margin_batch(orc):
    found = {}
    for sp in CF.batch_instances():
        bg = M.background_grid(sp["bg_n"], -2.0, 2.0, amp=0.02)
        axes = (0.5, 0.35, 0.25) if sp["kind"] == "ellipsoid" else None
        s = M.cube_sphere(sp["m"], R=0.5, axes=axes, dimples=sp["dimples"], dimple_a=CF.DIMPLE_A,
                          dimple_k=CF.DIMPLE_K)
        band, d = _near(orc, bg, s, np.asarray(sp["pose"], dtype=np.float64))
        _, near = _contacts(band, d)
        if near:
            found[sp["index"]] = near
    assert list(found) == [1] and len(found[1]) == 1
    assert abs(list(found[1].values())[0] - 3.18e-7) < 1e-9


@pytest.mark.slow
def test_margin_two_body(orc):
    two = CF.two_body()
    walls = [b["surface"] for b in two["bodies"]]
    sh = two["bodies"][0]["shell"]
    sh_boxes = PU.element_boxes(sh)
    exact, near_steps = {}, {}
    for step in (0, 1, 2, 3, 4, 5, 10, 37, 57, 100, 123, 199, 200, 250, 300, 399):
        poses = CF.two_body_poses(step)
        rel = PU.pose_compose(PU.pose_inverse(poses[0]), poses[1])
        band, d = _near(orc, sh, walls[1], rel, boxes=sh_boxes)
        n0, near = _contacts(band, d)
        if n0:
            exact[step] = n0
        if near:
            near_steps[step] = sorted(near.values())
    assert exact == {0: 4, 100: 4, 250: 4, 300: 4}
    assert sorted(near_steps) == [1, 2, 399]
    for step in (0, 37):
        for k, p in enumerate(CF.two_body_poses(step)):
            band, d = _near(orc, two["bg"], walls[k], p)
            _, near = _contacts(band, d)
            assert near == {}
