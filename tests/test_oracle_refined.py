"""Pins of the oracle's refined cut (the cut on the curved faces, reached by
splitting every quadratic face into k x k quadratic sub-faces and every
element into k^3 quadratic sub-elements, each the isoparametric map on a
sub-domain).

* Level 1 is the lattice cut, bit for bit.
* Flat faces on an undisplaced grid: refinement changes no geometry, so the
  refined cut equals the lattice cut and the closed-form box count.
* The refined surface stays closed: winding number 1 inside, 0 outside.
* Convergence: element-surface distances of levels k and 2k differ by no more
  than the stated linearisation bounds of the two levels (the refined
  triangulations lie within those bounds of the curved faces).
* A sphere: the distances of level 6 match the analytic distance to the
  sphere to within the bound plus the quadratic faces' own deviation from the
  sphere (measured on the inputs), much closer than level 1 does."""
import numpy as np
import pytest

from workloads import configs as CF
from workloads import meshes as M


def test_level_one_is_the_lattice_cut(orc):
    case = CF.tiny()
    bg, s = case["bg"], case["bodies"][0]["surface"]
    assert np.array_equal(orc.cut_surface_refined(bg, s, 1), orc.cut_surface(bg, s))
    rng = np.random.default_rng(5)
    bg = M.background_grid(10, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(4, R=0.5, dimples=12, dimple_a=0.1, dimple_k=0.03)
    pose = M.random_pose(rng, 0.2)
    assert np.array_equal(orc.cut_surface_refined(bg, s, 1, pose), orc.cut_surface(bg, s, pose))


def test_flat_faces_are_unchanged_by_refinement(orc):
    n, lo, hi = 10, -1.5, 1.5
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = (-0.41, 0.63, -0.2), (0.37, 0.88, 0.61)
    s = M.box_surface(2, a, b)
    base = orc.cut_surface(g, s)
    e = np.linspace(lo, hi, n + 1)
    cnt = [int(((e[1:] >= a[k]) & (e[:-1] <= b[k])).sum()) for k in range(3)]
    assert (base == 0).sum() == cnt[0] * cnt[1] * cnt[2]
    for k in (2, 3):
        assert np.array_equal(orc.cut_surface_refined(g, s, k), base)


@pytest.mark.parametrize("k", [2, 3])
def test_refined_surface_is_closed(orc, k):
    s = M.cube_sphere(4, R=0.5, dimples=10, dimple_a=0.1, dimple_k=0.03)
    sv = orc.refine_surface(s, k)
    assert sv.n_face == s.n_face * k * k
    tris = []
    for f in sv.conn:
        L = f.reshape(3, 3).T
        for m in range(2):
            for q in range(2):
                tris.append((L[m][q], L[m + 1][q], L[m + 1][q + 1]))
                tris.append((L[m][q], L[m + 1][q + 1], L[m][q + 1]))
    P = sv.nodes
    w_in = sum(orc.solid_angle(np.zeros(3), P[a], P[b], P[c]) for a, b, c in tris) / (4 * np.pi)
    w_out = sum(orc.solid_angle(np.array([0.8, 0.3, -0.1]), P[a], P[b], P[c]) for a, b, c in tris) / (4 * np.pi)
    assert abs(w_in - 1.0) < 1e-9 and abs(w_out) < 1e-9


def _element_faces9(grid, e):
    """The six 3x3 face lattices of element e (order -xi, +xi, -eta, +eta,
    -zeta, +zeta; lattice index a + 3b in the face's own axes)."""
    X = grid.nodes[grid.conn[e]].reshape(3, 3, 3, 3)       # [c, b, a]
    return [X[:, :, 0].reshape(9, 3), X[:, :, 2].reshape(9, 3), X[:, 0, :].reshape(9, 3),
            X[:, 2, :].reshape(9, 3), X[0].reshape(9, 3), X[2].reshape(9, 3)]


def _distances(orc, grid, surf, k, pose, elems):
    sv = orc.refine_surface(surf, k)
    sub = orc.refine_elements(grid, elems, k)
    d = orc.cut_surface(sub, sv, pose, diagnostics=True)["dstar"]
    return d.reshape(len(elems), k ** 3).min(axis=1)


def test_refinement_converges_within_its_bound(orc):
    bg = M.background_grid(8, -1.0, 1.0, amp=0.05)
    s = M.cube_sphere(3, R=0.5, dimples=8, dimple_a=0.12, dimple_k=0.04)
    pose = M.IDENTITY_POSE
    elems = np.arange(bg.n_elem)
    eps_s = {k: max(orc.refinement_bound(s.nodes[f], k) for f in s.conn) for k in (1, 2, 4)}
    eps_e = {k: np.array([max(orc.refinement_bound(F, k) for F in _element_faces9(bg, e)) for e in elems])
             for k in (1, 2, 4)}
    d = {k: _distances(orc, bg, s, k, pose, elems) for k in (1, 2, 4)}
    assert eps_s[1] > 4 * eps_s[2] * 0.99 and eps_s[2] > 4 * eps_s[4] * 0.99      # O(1 / k^2)
    for k in (1, 2):
        slack = eps_s[k] + eps_s[2 * k] + eps_e[k] + eps_e[2 * k]
        away = (d[k] > 0) & (d[2 * k] > 0)
        assert away.sum() > 100
        assert np.all(np.abs(d[k][away] - d[2 * k][away]) <= slack[away] + 1e-12)
    # the lattice level is visibly farther from the finest level than level 2
    assert np.abs(d[1] - d[4]).max() > 2 * np.abs(d[2] - d[4]).max()


def test_sphere_distances_approach_the_analytic_ones(orc):
    R = 0.5
    s = M.cube_sphere(3, R=R)
    bg = M.background_grid(10, -1.0, 1.0, amp=0.0)
    P = bg.nodes[bg.conn]
    lo, hi = P.min(axis=1), P.max(axis=1)
    near = np.clip(0.0, lo, hi)                               # the box point nearest the centre
    far = np.sqrt((np.maximum(np.abs(lo), np.abs(hi)) ** 2).sum(axis=1))
    rmin = np.linalg.norm(near, axis=1)
    outside = np.nonzero((rmin > R + 0.02) & (rmin < R + 0.3))[0]
    inside = np.nonzero(far < R - 0.02)[0]
    outside, inside = outside[::4], inside[::2]
    elems = np.concatenate([outside, inside])
    d_an = np.concatenate([rmin[outside] - R, R - far[inside]])
    # deviation of the quadratic faces from the sphere, measured on the inputs
    u = np.linspace(-1, 1, 41)
    L = np.stack([0.5 * u * (u - 1), 1 - u * u, 0.5 * u * (u + 1)], axis=1)
    dev = 0.0
    for f in s.conn:
        X = s.nodes[f].reshape(3, 3, 3)
        pts = np.einsum("bax,ia,jb->ijx", X, L, L)
        dev = max(dev, np.abs(np.linalg.norm(pts, axis=2) - R).max())
    eps6 = max(orc.refinement_bound(s.nodes[f], 6) for f in s.conn)
    d1 = _distances(orc, bg, s, 1, M.IDENTITY_POSE, elems)
    d6 = _distances(orc, bg, s, 6, M.IDENTITY_POSE, elems)
    assert elems.size > 40
    assert np.all(np.abs(d6 - d_an) <= eps6 + dev + 1e-12)
    assert np.abs(d1 - d_an).max() > 3 * np.abs(d6 - d_an).max()
