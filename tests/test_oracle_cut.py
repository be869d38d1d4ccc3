"""Pins of the oracle's direct cut: closed-form box and sphere cuts, brute
force on small grids, invariants (no GPU)."""
import math

import numpy as np
import pytest

from workloads import meshes as M
from workloads import configs as CF


def _cells(n, lo, hi):
    e = np.linspace(lo, hi, n + 1)
    return e[:-1], e[1:]


def test_box_cut_closed_form(orc):
    """Axis-aligned box of flat quads on an undisplaced grid: the holes are
    exactly the cells meeting the closed box, and the fringe is the one-cell
    face layer around that block."""
    n, lo, hi = 12, -1.5, 1.5
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = (-0.41, 0.63, -0.2), (0.37, 0.88, 0.61)
    s = M.box_surface(3, a, b)
    ib = orc.cut(g, [s], [orc.IDENTITY])
    l, u = _cells(n, lo, hi)
    cnt, rng_ = [], []
    for ax in range(3):
        m = (u >= a[ax]) & (l <= b[ax])
        cnt.append(int(m.sum()))
        rng_.append(np.nonzero(m)[0])
    assert (ib == orc.HOLE).sum() == cnt[0] * cnt[1] * cnt[2]
    nx, ny, nz = cnt
    assert (ib == orc.FRINGE).sum() == 2 * (nx * ny + ny * nz + nx * nz)
    e = np.arange(n ** 3)
    i, j, k = e % n, (e // n) % n, e // n ** 2
    inblock = np.isin(i, rng_[0]) & np.isin(j, rng_[1]) & np.isin(k, rng_[2])
    assert np.all((ib == orc.HOLE) == inblock)


def test_box_cut_overset_keeps_cut_cells(orc):
    """Overset kind: cells cut by the surface stay field; only cells strictly
    inside become holes."""
    n, lo, hi = 10, -1.0, 1.0
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = (-0.55, -0.33, -0.71), (0.45, 0.5, 0.29)
    s = M.box_surface(2, a, b)
    st = orc.cut_surface(g, s, kind=orc.SURF_OVERSET)
    l, u = _cells(n, lo, hi)
    cnt = [int(((l > a[ax]) & (u < b[ax])).sum()) for ax in range(3)]
    assert (st == 0).sum() == cnt[0] * cnt[1] * cnt[2]


def _sphere_bounds(n, lo, hi, surf, R):
    l, u = _cells(n, lo, hi)
    e = np.arange(n ** 3)
    idx = [e % n, (e // n) % n, e // n ** 2]
    near2 = np.zeros(n ** 3)
    far2 = np.zeros(n ** 3)
    for ax in range(3):
        lo_, hi_ = l[idx[ax]], u[idx[ax]]
        c = np.clip(0.0, lo_, hi_)
        near2 += c * c
        far2 += np.maximum(lo_ * lo_, hi_ * hi_)
    return np.sqrt(near2), np.sqrt(far2)


def _inradius(orc, surf):
    P = surf.nodes[surf.conn]
    best = np.inf
    for f in range(P.shape[0]):
        for n in range(2):
            for m in range(2):
                p00, p10, p11, p01 = P[f, m + 3 * n], P[f, m + 1 + 3 * n], P[f, m + 1 + 3 * (n + 1)], P[f, m + 3 * (n + 1)]
                for T in ((p00, p10, p11), (p00, p11, p01)):
                    d, _, _ = orc.tri_tri(np.stack(T), np.zeros((3, 3)))
                    best = min(best, d)
    return best


def test_sphere_bounds_undisplaced(orc):
    """Every vertex of the linearised sphere lies at R and every triangle at
    least r_in from the centre: cells closer than r_in are holes, cells beyond
    R are field, cells spanning both radii are hit, cells inside r_in are
    holes without a hit."""
    n, lo, hi, R = 14, -1.0, 1.0, 0.45
    g = M.background_grid(n, lo, hi, amp=0.0)
    s = M.cube_sphere(3, R=R)
    rin = _inradius(orc, s)
    assert 0.4 < rin < R
    r = orc.cut_surface(g, s, diagnostics=True)
    near, far = _sphere_bounds(n, lo, hi, s, R)
    hole = r["status"] == 0
    assert np.all(hole[near < rin])
    assert np.all(~hole[near > R])
    assert np.all(r["hit"][(near < rin) & (far > R)] == 1)
    assert np.all((r["hit"] == 0)[far < rin])
    assert (near < rin).sum() <= hole.sum() <= (near <= R).sum()


def test_tiny_case_counts(orc):
    """The tiny case is degenerate on purpose: the displacement vanishes on the
    coordinate planes, so background nodes (+-0.5,0,0), (0,+-0.5,0),
    (0,0,+-0.5) coincide with cube-sphere vertices and 24 elements touch the
    surface at distance exactly 0.  Expected: 8 cells strictly inside, 56
    crossing, 24 touching -> 88 holes, 96 fringe."""
    c = CF.tiny()
    bg, s = c["bg"], c["bodies"][0]["surface"]
    r = orc.cut_surface(bg, s, diagnostics=True)
    hit = r["hit"] == 1
    inside = (r["wind"] > 0.5) & ~hit
    assert inside.sum() == 8
    assert hit.sum() == 80
    ib = orc.cut(bg, [s], [orc.IDENTITY])
    assert (ib == orc.HOLE).sum() == 88
    assert (ib == orc.FRINGE).sum() == 96
    # central inversion symmetry of the tiny case: element (i,j,k) <-> (15-i,15-j,15-k)
    e = np.arange(16 ** 3)
    i, j, k = e % 16, (e // 16) % 16, e // 256
    inv = (15 - i) + 16 * (15 - j) + 256 * (15 - k)
    assert np.array_equal(ib, ib[inv])


def _small_case(seed, n=6, m=2):
    rng = np.random.default_rng(seed)
    g = M.background_grid(n, -0.8, 0.8, amp=0.05)
    s = M.cube_sphere(m, R=0.42, dimples=12, dimple_a=0.1, dimple_k=0.03)
    return g, s, M.random_pose(rng, 0.15), rng


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_equals_accelerated(orc, seed):
    """All-pairs (no pruning, no hierarchy) against the accelerated oracle."""
    g, s, pose, _ = _small_case(seed)
    rb = orc.cut_surface(g, s, pose, brute=True, diagnostics=True)
    ra = orc.cut_surface(g, s, pose, brute=False, diagnostics=True)
    assert np.array_equal(rb["status"], ra["status"])
    assert np.array_equal(rb["hit"], ra["hit"])
    assert np.array_equal(rb["nsign"], ra["nsign"])
    assert np.array_equal(rb["psign"], ra["psign"])
    np.testing.assert_allclose(rb["dstar"], ra["dstar"], rtol=0, atol=0)
    assert 0 < (ra["status"] == 0).sum() < g.n_elem


def test_nearest_sign_agrees_with_winding(orc):
    """Nearest-face side (Sec. 4.1/4.2 rule) equals the winding-number side on
    every non-hit element of the tiny case and a dimpled case."""
    c = CF.tiny()
    cases = [(c["bg"], c["bodies"][0]["surface"], orc.IDENTITY)]
    g = M.background_grid(20, -0.9, 0.9, amp=0.03)
    s = M.cube_sphere(8, R=0.5, dimples=40, dimple_a=0.08, dimple_k=0.02)
    cases.append((g, s, M.pose_rz(0.3, (0.02, -0.01, 0.03))))
    for g, s, p in cases:
        r = orc.cut_surface(g, s, p, diagnostics=True)
        nh = r["hit"] == 0
        assert np.array_equal(r["nsign"][nh] < 0, r["wind"][nh] > 0.5)
        assert np.array_equal(r["psign"][nh] < 0, r["wind"][nh] > 0.5)
        assert np.all(np.abs(r["wind"][nh] - np.round(r["wind"][nh])) < 1e-9)


def test_rigid_pose_invariance(orc):
    """iblank is unchanged when grid and surface move together."""
    g, s, pose, rng = _small_case(3, n=8, m=3)
    ib0 = orc.cut(g, [s], [pose])
    Q = M.random_pose(rng, 0.5)
    g2 = M.Grid(nodes=M.apply_pose_to_points(Q, g.nodes), conn=g.conn)
    ib1 = orc.cut(g2, [s], [M.compose_pose(Q, pose)])
    assert np.array_equal(ib0, ib1)


def test_relabeling_and_union(orc):
    g, s, pose, rng = _small_case(4, n=8, m=3)
    st = orc.cut_surface(g, s, pose)
    perm = rng.permutation(g.n_elem)
    g2 = M.Grid(nodes=g.nodes, conn=g.conn[perm])
    assert np.array_equal(orc.cut_surface(g2, s, pose), st[perm])
    fperm = rng.permutation(s.n_face)
    s2 = M.Surface(nodes=s.nodes, conn=s.conn[fperm])
    assert np.array_equal(orc.cut_surface(g, s2, pose), st)
    # union of two surfaces is the elementwise union of holes
    s3 = M.cube_sphere(2, R=0.2)
    p3 = M.pose_rz(0.0, (0.45, 0.4, -0.3))
    st3 = orc.cut_surface(g, s3, p3)
    nbr = orc.face_neighbors(g.conn)
    ib = orc.cut(g, [s, s3], [pose, p3], nbr=nbr)
    assert np.array_equal(ib == orc.HOLE, (st == 0) | (st3 == 0))


def test_element_winding_and_enclosed_surface(orc):
    """The element boundary is a closed surface: winding 1 at interior points
    (positive Jacobian), 0 outside; a surface lying inside one element makes
    that element hit."""
    g = M.background_grid(1, -1.0, 1.0, amp=0.0)
    g.nodes[:] += 0.07 * np.sin(3.0 * g.nodes[:, [1, 2, 0]])
    for p, w in (([0.05, -0.1, 0.2], 1.0), ([0.7, 0.6, -0.65], 1.0), ([1.6, 0, 0], 0.0), ([0, -2, 0.3], 0.0)):
        assert orc.element_winding(g.nodes, g.conn, 0, p) == pytest.approx(w, abs=1e-12)
    s = M.cube_sphere(2, R=0.3)
    r = orc.cut_surface(g, s, diagnostics="point")
    assert r["hit"][0] == 1 and r["status"][0] == 0
    assert orc.cut_surface(g, s, kind=orc.SURF_OVERSET)[0] == 1
