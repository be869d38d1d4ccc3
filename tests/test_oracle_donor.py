"""Pins of the oracle's receptor points and donor search (no GPU)."""
import math

import numpy as np
import pytest

from workloads import meshes as M
from workloads import configs as CF


def test_fringe_points_affine_grid(orc):
    """On an undisplaced grid the Gauss points are closed-form."""
    g = M.background_grid(4, -1.0, 1.0, amp=0.0)
    e = np.array([0, 5, 63])
    pts = orc.fringe_points(g, e)
    gp = math.sqrt(0.6)
    h = 0.5
    for q, el in enumerate(e):
        i, j, k = el % 4, (el // 4) % 4, el // 16
        c = -1.0 + h * (np.array([i, j, k]) + 0.5)
        for cc in range(3):
            for b in range(3):
                for a in range(3):
                    exp = c + 0.5 * h * np.array([(a - 1) * gp, (b - 1) * gp, (cc - 1) * gp])
                    np.testing.assert_allclose(pts[27 * q + a + 3 * b + 9 * cc], exp, atol=1e-15)


def test_self_donor(orc):
    """A curved grid's own Gauss points are found in their own elements."""
    g = M.background_grid(5, -1.0, 1.0, amp=0.04)
    rng = np.random.default_rng(0)
    e = np.sort(rng.choice(g.n_elem, 20, replace=False))
    pts = orc.fringe_points(g, e)
    donor, xi, _ = orc.donor_search(g, pts)
    assert np.array_equal(donor, np.repeat(e, 27).astype(np.int32))
    gp = math.sqrt(0.6)
    ref = np.array([[(a - 1) * gp, (b - 1) * gp, (c - 1) * gp]
                    for c in range(3) for b in range(3) for a in range(3)])
    np.testing.assert_allclose(xi, np.tile(ref, (20, 1)), atol=1e-12)


def test_donors_brute_force_and_invariants(orc):
    """Tiny case, both directions: the accelerated search equals the all-element
    search; donors reproduce their points; reference coordinates lie in
    [-1, 1]^3; orphans have no containing element at all."""
    c = CF.tiny()
    bg, s, sh = c["bg"], c["bodies"][0]["surface"], c["bodies"][0]["shell"]
    ib = orc.cut(bg, [s], [orc.IDENTITY])
    pts_bg = orc.fringe_points(bg, orc.fringe_elements(ib))
    ish = orc.cut(sh, [], [])
    assert (ish == orc.FRINGE).sum() == 96
    pts_sh = orc.fringe_points(sh, orc.fringe_elements(ish))
    rng = np.random.default_rng(1)
    for grid, pts in ((sh, pts_bg), (bg, pts_sh[rng.choice(pts_sh.shape[0], 400, replace=False)])):
        d, xi, info = orc.donor_search(grid, pts)
        db, xib, _ = orc.donor_search(grid, pts, brute=True)
        assert np.array_equal(d, db)
        ok = d >= 0
        np.testing.assert_allclose(xi[ok], xib[ok], atol=0)
        assert np.all(np.abs(xi[ok]) <= 1 + 1e-10)
        assert np.all(np.isnan(xi[~ok]))
        for i in np.nonzero(ok)[0][:200]:
            X = grid.nodes[grid.conn[d[i]]]
            x, _ = orc.q2_eval(X, xi[i])
            diam = np.linalg.norm(X.max(0) - X.min(0))
            assert np.linalg.norm(x - pts[i]) <= 1e-12 * diam
    # bg -> shell: orphans lie outside the shell's radial range [0.5, 1]
    # (beyond its outer boundary, or between the linearised cut surface and
    # the curved inner wall)
    d, _, _ = orc.donor_search(sh, pts_bg)
    r = np.linalg.norm(pts_bg, axis=1)
    assert np.all((r[d < 0] < 0.5) | (r[d < 0] > 0.99))
    assert np.all(d[(r > 0.51) & (r < 0.98)] >= 0)
    assert 0 < (d < 0).sum() < 100


def test_donor_pose_consistency(orc):
    """Searching posed points in a posed grid equals searching the unposed
    points in the unposed grid (the rigid-motion search of Sec. 4.3)."""
    g = M.background_grid(5, -1.0, 1.0, amp=0.04)
    rng = np.random.default_rng(2)
    pts = rng.uniform(-0.95, 0.95, (300, 3))
    d0, xi0, _ = orc.donor_search(g, pts)
    Q = M.random_pose(rng, 0.4)
    d1, xi1, _ = orc.donor_search(g, M.apply_pose_to_points(Q, pts), pose=Q)
    assert np.array_equal(d0, d1)
    np.testing.assert_allclose(xi0, xi1, atol=1e-12)
