"""Pins of the oracle's filtered cut, the paper's own pipeline (Sec. 4.2,
Alg. cp0, bboxdix, cp1, cp2): box distance in closed form, element OBBs of
axis-aligned and rotated boxes, agreement with the closed-form box cut, and
the property that a truncation can only lose, never invent, intersections
(no GPU)."""
import numpy as np

from workloads import meshes as M


def test_bbox_dist_closed_form(orc):
    a = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    assert orc.hx_bbox_dist(a, [1.5, 0.2, 0.3, 2.0, 0.8, 0.9]) == 0.5          # apart along x only
    assert orc.hx_bbox_dist([-2.0, 0.1, 0.1, -1.0, 0.9, 0.9], a) == 1.0      # order of the boxes
    assert abs(orc.hx_bbox_dist(a, [1.3, 1.4, -5.0, 2.0, 2.0, 5.0]) - 0.5) <= 1e-16   # x and y: 0.3, 0.4
    assert abs(orc.hx_bbox_dist(a, [-3.0, -3.0, -3.0, -2.0, -2.0, -2.0]) - np.sqrt(3.0) * 2.0) <= 1e-15
    assert orc.hx_bbox_dist(a, [0.5, 0.5, 0.5, 3.0, 3.0, 3.0]) == 0.0        # overlapping
    assert orc.hx_bbox_dist(a, [1.0, 0.0, 0.0, 2.0, 1.0, 1.0]) == 0.0        # touching


def _box_element(lo, hi, R=np.eye(3)):
    """27 lattice nodes of a box element (node a + 3b + 9c), rotated by R."""
    X = np.empty((27, 3))
    for k in range(27):
        a, b, c = k % 3, (k // 3) % 3, k // 9
        X[k] = [lo[0] + (hi[0] - lo[0]) * a / 2, lo[1] + (hi[1] - lo[1]) * b / 2, lo[2] + (hi[2] - lo[2]) * c / 2]
    return X @ R.T


def test_obb_of_boxes(orc):
    """An axis-aligned box element's OBB is the box itself; a rotated one's
    axes are the rotated coordinate axes (up to order and sign) and its
    extents the box's edge lengths; the centroid is the box centre."""
    lo, hi = np.array([0.1, -0.4, 0.25]), np.array([0.6, 0.3, 0.45])   # distinct edges: no repeated eigenvalue
    cg, R, B = orc.hx_obb(_box_element(lo, hi))
    assert np.abs(cg - 0.5 * (lo + hi)).max() <= 1e-15
    assert np.abs(R - np.eye(3)).max() <= 1e-15
    assert np.abs(B - np.concatenate([lo, hi])).max() <= 1e-15
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    Q = Q @ np.array([[1.0, 0.0, 0.0], [0.0, np.cos(0.4), -np.sin(0.4)], [0.0, np.sin(0.4), np.cos(0.4)]])
    cg, R, B = orc.hx_obb(_box_element(lo, hi, Q))
    assert np.abs(R @ R.T - np.eye(3)).max() <= 1e-14
    # each OBB axis is (up to sign) one rotated coordinate axis
    A = np.abs(R @ Q)
    assert np.abs(np.sort(A, axis=1)[:, -1] - 1.0).max() <= 1e-12
    assert np.abs(np.sort(B[3:] - B[:3]) - np.sort(hi - lo)).max() <= 1e-12
    assert np.abs(cg - Q @ (0.5 * (lo + hi))).max() <= 1e-14


def _cells(n, lo, hi):
    e = np.linspace(lo, hi, n + 1)
    return e[:-1], e[1:]


def test_box_cut_matches_closed_form(orc):
    """A box wall on an undisplaced grid: the filtered cut (N_F^1 = 16,
    N_F^2 = 4, and the extreme truncation 1, 1) gives the cells meeting the
    box, with one fringe layer, as the plain definition does."""
    n, lo, hi = 12, -1.2, 1.2
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = np.array([-0.41, -0.33, -0.27]), np.array([0.36, 0.52, 0.31])
    s = M.box_surface(2, a, b)
    l, u = _cells(n, lo, hi)
    e = np.arange(n ** 3)
    idx = [e % n, (e // n) % n, e // n ** 2]
    want = np.ones(n ** 3, dtype=bool)
    for ax in range(3):
        want &= ((u >= a[ax]) & (l <= b[ax]))[idx[ax]]
    exact = orc.cut(g, [s], [M.IDENTITY_POSE])
    assert np.array_equal(exact == orc.HOLE, want)
    for nf1, nf2 in ((16, 4), (1, 1)):
        assert np.array_equal(orc.cut_heuristic(g, [s], [M.IDENTITY_POSE], nf1=nf1, nf2=nf2), exact)


def test_truncation_never_invents_a_hit(orc):
    """A second-pass hit is an exact triangle pair below the tolerance, so
    every element the filtered cut finds intersected is intersected under the
    plain definition; with the paper's N_F^1 = 16, N_F^2 = 4 no element of
    the dimpled case is missed."""
    g = M.background_grid(12, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(5, R=0.5, dimples=20, dimple_a=0.09, dimple_k=0.03)
    p = M.pose_rz(0.3, (0.05, 0.0, 0.0))
    ex = orc.cut_surface(g, s, p, diagnostics="point")
    for nf1, nf2 in ((16, 4), (2, 1), (1, 1)):
        st, hit = orc.cut_surface_heuristic(g, s, p, nf1=nf1, nf2=nf2)
        assert np.all(ex["hit"][hit == 1] == 1), (nf1, nf2)
        if (nf1, nf2) == (16, 4):
            assert np.array_equal(hit, ex["hit"]) and np.array_equal(st, ex["status"])
    # the extreme truncation does lose holes here (the ablation has something to measure)
    st11, _ = orc.cut_surface_heuristic(g, s, p, nf1=1, nf2=1)
    assert (st11 != ex["status"]).sum() > 0


def test_overset_kind(orc):
    """Overset surfaces: intersected elements stay field; the rest of the
    filtered cut is unchanged."""
    g = M.background_grid(10, -1.0, 1.0, amp=0.03)
    s = M.cube_sphere(4, R=0.5)
    st_w, hit = orc.cut_surface_heuristic(g, s, M.IDENTITY_POSE, kind=orc.SURF_WALL)
    st_o, hit_o = orc.cut_surface_heuristic(g, s, M.IDENTITY_POSE, kind=orc.SURF_OVERSET)
    assert np.array_equal(hit, hit_o) and hit.sum() > 0
    assert np.all(st_o[hit == 1] == 1) and np.all(st_w[hit == 1] == 0)
    assert np.array_equal(st_o[hit == 0], st_w[hit == 0])
    assert np.array_equal(st_o, orc.cut_surface(g, s, M.IDENTITY_POSE, kind=orc.SURF_OVERSET))


def _flat_quad(centre, half, z_axis=2):
    """One 9-node flat square face of half-width ``half`` normal to the
    given axis, centred at ``centre``."""
    u, v = [k for k in range(3) if k != z_axis]
    P = np.empty((9, 3))
    for k in range(9):
        a, b = k % 3, k // 3
        P[k] = centre
        P[k, u] += (a - 1) * half
        P[k, v] += (b - 1) * half
    return P


class _Faces:
    def __init__(self, quads):
        self.nodes = np.concatenate(quads)
        self.conn = np.arange(9 * len(quads), dtype=np.int32).reshape(-1, 9)


def test_approx_distance_and_pass1_ranking(orc):
    """Alg. cp0 ranks by box distance in the element's OBB frame plus 1/100
    of the centroid distance: two faces inside the element's box rank by
    their centroids; Alg. cp1 keeps the faces by their linear distance and
    the corner nearest each face's centroid."""
    X = _box_element([0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    quads = [_flat_quad([0.2, 0.2, 0.2], 0.05),      # 0: inside, 0.52 from the centre
             _flat_quad([0.5, 0.5, 1.7], 0.05),      # 1: above, box gap 0.7
             _flat_quad([0.55, 0.5, 0.5], 0.05),     # 2: inside, 0.05 from the centre
             _flat_quad([1.3, 0.5, 0.5], 0.05, 0)]   # 3: beside, box gap 0.3
    l1, d1, l2, d2, c2 = orc.hx_lists(X, _Faces(quads), nf1=4, nf2=2)
    assert list(l1) == [2, 0, 3, 1]
    assert abs(d1[0] - 0.01 * 0.05) <= 1e-15
    assert abs(d1[1] - 0.01 * np.sqrt(3 * 0.3 ** 2)) <= 1e-15
    assert abs(d1[2] - (0.3 + 0.01 * 0.8)) <= 1e-15
    assert abs(d1[3] - (0.7 + 0.01 * 1.2)) <= 1e-15
    # first pass, over the three element faces at the corner nearest each
    # face centroid: face 0 -> corner 0, 0.15 from x = 0 (and y = 0); face 2
    # -> corner 1 (the first of the four equally near x = 1 corners), 0.4
    # from x = 1; face 3 -> corner 1, 0.3 from x = 1; face 1 -> 0.7
    assert list(l2) == [0, 3]
    assert abs(d2[0] - 0.15) <= 1e-15 and c2[0] == 0
    assert abs(d2[1] - 0.3) <= 1e-15 and c2[1] == 1
    l1, d1, l2, d2, c2 = orc.hx_lists(X, _Faces(quads), nf1=4, nf2=4)
    assert list(l2) == [0, 3, 2, 1] and abs(d2[2] - 0.4) <= 1e-15 and c2[2] == 1


def test_pass1_uses_the_faces_at_the_nearest_corner(orc):
    """Six small faces, each 0.05 inside one face of the unit box element and
    pulled towards a corner of that face: each is nearest to that corner, and
    the first pass finds its 0.05 gap through the element face at the corner
    (any other face is at least 0.25 away)."""
    X = _box_element([0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    spec = [((0.05, 0.3, 0.3), 0, 0),    # -xi face, corner (0,0,0) = 0
            ((0.95, 0.7, 0.7), 0, 7),    # +xi face, corner (1,1,1) = 7
            ((0.3, 0.05, 0.7), 1, 4),    # -eta face, corner (0,0,1) = 4
            ((0.7, 0.95, 0.3), 1, 3),    # +eta face, corner (1,1,0) = 3
            ((0.7, 0.3, 0.05), 2, 1),    # -zeta face, corner (1,0,0) = 1
            ((0.3, 0.7, 0.95), 2, 6)]    # +zeta face, corner (0,1,1) = 6
    quads = [_flat_quad(np.array(c), 0.05, ax) for c, ax, _ in spec]
    l1, d1, l2, d2, c2 = orc.hx_lists(X, _Faces(quads), nf1=6, nf2=6)
    got = {int(f): (d, int(c)) for f, d, c in zip(l2, d2, c2)}
    for f, (_, _, corner) in enumerate(spec):
        d, c = got[f]
        assert c == corner, (f, c)
        assert abs(d - 0.05) <= 1e-15, (f, d)
