"""Oracle pins on the connectivity-robustness cases (Sec. 4.4: a slot
through the body, a groove, rotated and anisotropic backgrounds; Sec. 4.1,
Fig. multinorm: equidistant faces whose normals must or must not be
averaged).

* Input margin: every element is intersected (distance 0) or at least 1e-6
  from the surface, so the 1e-7 hit threshold is decided alike in any FP64
  operation order.
* The nearest-face side of each non-hit element (element pair, and first
  node, with the tie rule) equals the side of the winding number, on
  geometry built to make the tie rule decide.
* The unposed slotted plate on an undisplaced grid: hole count in closed
  form (elements whose closed box meets a solid cell of the plate).
* The wedge: its construction puts element 942's first node in the
  averaging branch of the tie rule (checked from the geometry alone), and
  the oracle places that element outside."""
import numpy as np
import pytest

import robust_cases as RC
from workloads import meshes as M


@pytest.mark.parametrize("name", RC.NAMES)
def test_margin_and_side_rule(orc, name):
    bg, s, pose = RC.case(name)
    d = orc.cut_surface(bg, s, pose, diagnostics=True)
    ds = d["dstar"]
    fragile = np.nonzero((ds > 0) & (ds < 1e-6))[0]
    assert fragile.size == 0, "%s: elements within (0, 1e-6) of the surface: %s" % (name, fragile[:8])
    nonhit = d["hit"] == 0
    assert nonhit.sum() > 0 and (~nonhit).sum() > 0
    side_w = np.where(d["wind"] > 0.5, -1, 1)
    assert np.all(np.abs(d["wind"] - np.round(d["wind"])) < 1e-9), "winding numbers must be integers"
    assert np.array_equal(d["psign"][nonhit], side_w[nonhit])
    assert np.array_equal(d["nsign"][nonhit], side_w[nonhit])


def test_slotted_plate_closed_form(orc):
    bg = M.background_grid(12, -1.5, 1.5, amp=0.0)
    s = M.slotted_plate(w=0.4, c=0.35)
    ib = orc.cut(bg, [s], [M.IDENTITY_POSE])
    xs, ys, zs = s.meta["xs"], s.meta["ys"], s.meta["zs"]
    P = bg.nodes[bg.conn]
    lo, hi = P.min(axis=1), P.max(axis=1)
    hole = np.zeros(bg.n_elem, dtype=bool)
    for i in range(3):
        for j in range(3):
            if i == 1 and j == 1:
                continue          # the slot
            cell_lo = np.array([xs[i], ys[j], zs[0]])
            cell_hi = np.array([xs[i + 1], ys[j + 1], zs[1]])
            hole |= np.all(hi >= cell_lo, axis=1) & np.all(lo <= cell_hi, axis=1)
    assert np.array_equal(ib == orc.HOLE, hole)
    # the elements inside the slot, clear of its walls, stay field or fringe
    inner = np.all(lo > [-0.4, -0.5, -2], axis=1) & np.all(hi < [0.4, 0.5, 2], axis=1)
    assert inner.sum() > 0 and np.all(ib[inner] != orc.HOLE)


def test_wedge_takes_the_averaging_branch(orc):
    bg, s, pose = RC.case("wedge")
    m = s.meta
    p = bg.nodes[bg.conn[RC.WEDGE_ELEMENT, 0]]
    assert np.array_equal(p, np.zeros(3))
    # the apex edge is the nearest feature; its two faces' outward normals
    n1 = m["n0"] + m["t"] * m["b"]
    n2 = -m["n0"] + m["t"] * m["b"]
    n1 /= np.linalg.norm(n1)
    n2 /= np.linalg.norm(n2)
    v = p - m["apex"]
    assert abs(v @ m["e"]) < 1e-15 and abs(np.linalg.norm(v) - RC.WEDGE_DELTA) < 1e-15
    v /= np.linalg.norm(v)
    # inside the edge's normal cone (v = a n1 + b n2 with a, b >= 0)
    a_, b_ = np.linalg.lstsq(np.stack([n1, n2], axis=1), v, rcond=None)[0]
    assert a_ > 0 and b_ > 0
    d1, d2 = v @ n1, v @ n2
    assert d1 > 0 > d2, "opposite signs"
    assert 0 < abs(d1) - abs(d2) < 1e-9, "within the tie tolerance: %g" % (abs(d1) - abs(d2))
    assert v @ (n1 + n2) > 0     # the averaged normal: outside
    d = orc.cut_surface(bg, s, pose, sel=np.array([RC.WEDGE_ELEMENT]), diagnostics=True)
    assert d["hit"][0] == 0 and abs(d["dstar"][0] - RC.WEDGE_DELTA) < 1e-12
    assert d["psign"][0] == 1 and abs(d["wind"][0]) < 1e-9 and d["status"][0] == 1
