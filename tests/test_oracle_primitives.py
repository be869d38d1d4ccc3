"""Pins of the oracle's geometric and isoparametric primitives against closed
forms, brute force and invariants (no GPU)."""
import math

import numpy as np
import pytest


def _rand_tri(rng, c=0.0, s=1.0):
    return c + s * rng.standard_normal((3, 3))


# ---------------------------------------------------------------- tri-tri --

def test_tri_tri_parallel_offset(orc):
    A = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    B = A + np.array([0.1, 0.1, 0.37])
    d, pa, pb = orc.tri_tri(A, B)
    assert d == pytest.approx(0.37, abs=1e-15)
    assert np.linalg.norm(pa - pb) == pytest.approx(d, abs=1e-15)


def test_tri_tri_crossing_is_zero(orc):
    A = np.array([[-1, -1, 0], [2, -1, 0], [-1, 2, 0]], float)
    B = np.array([[0.2, 0.2, -1], [0.3, 0.25, 1], [0.25, 0.4, 1]], float)   # pierces A
    d, _, _ = orc.tri_tri(A, B)
    assert d == 0.0


def test_tri_tri_shared_vertex_exact_zero(orc):
    A = np.array([[0.5, 0, 0], [1, 0, 0], [0.5, 1, 0]], float)
    B = np.array([[0.5, 0, 0], [0, -1, 1], [0, -1, -1]], float)
    d, _, _ = orc.tri_tri(A, B)
    assert d == 0.0


def test_tri_tri_vertex_face(orc):
    A = np.array([[0, 0, 0], [4, 0, 0], [0, 4, 0]], float)
    B = np.array([[1, 1, 0.25], [1, 1, 3], [2, 1.5, 3]], float)   # apex above A's interior
    d, pa, pb = orc.tri_tri(A, B)
    assert d == pytest.approx(0.25, abs=1e-15)
    np.testing.assert_allclose(pa, [1, 1, 0], atol=1e-15)


def test_tri_tri_edge_edge_skew(orc):
    # edge of A along x at z=0, edge of B along y at height h: distance h
    h = 0.3
    A = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, -2]], float)
    B = np.array([[0, -1, h], [0, 1, h], [0.5, 0, 3]], float)
    d, pa, pb = orc.tri_tri(A, B)
    assert d == pytest.approx(h, abs=1e-15)
    np.testing.assert_allclose(pa, [0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(pb, [0, 0, h], atol=1e-15)


def test_tri_tri_symmetric_and_bounded_by_sampling(orc):
    rng = np.random.default_rng(5)
    w = np.array([(i, j) for i in range(41) for j in range(41 - i)], float) / 40.0
    bary = np.stack([1 - w.sum(1), w[:, 0], w[:, 1]], axis=1)
    for _ in range(40):
        A = _rand_tri(rng)
        B = _rand_tri(rng, c=rng.uniform(-1.5, 1.5), s=0.8)
        d1, pa, pb = orc.tri_tri(A, B)
        d2, _, _ = orc.tri_tri(B, A)
        assert d1 == pytest.approx(d2, rel=1e-12, abs=1e-14)
        # the returned points lie on the triangles and realise d
        assert np.linalg.norm(pa - pb) == pytest.approx(d1, rel=1e-12, abs=1e-14)
        PA = bary @ A
        PB = bary @ B
        # sampled distance is an upper bound that converges to d
        best = np.inf
        for k in range(0, PA.shape[0], 200):
            diff = PA[k:k + 200, None, :] - PB[None, :, :]
            best = min(best, np.sqrt((diff ** 2).sum(-1)).min())
        assert d1 <= best + 1e-12
        assert best - d1 <= 0.12


# ---------------------------------------------------------- solid angle --

def test_solid_angle_octant(orc):
    om = orc.solid_angle([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1])
    assert om == pytest.approx(math.pi / 2, rel=1e-14)


def test_winding_of_closed_box(orc):
    from workloads import meshes as M
    s = M.box_surface(2, -0.5, 0.5)
    tris = []
    for f in s.conn:
        P = s.nodes[f]
        for n in range(2):
            for m in range(2):
                p00, p10, p11, p01 = P[m + 3 * n], P[m + 1 + 3 * n], P[m + 1 + 3 * (n + 1)], P[m + 3 * (n + 1)]
                tris += [(p00, p10, p11), (p00, p11, p01)]
    for p, w in (([0.1, -0.2, 0.3], 1.0), ([0.7, 0, 0], 0.0), ([0.2, 0.2, -2.0], 0.0)):
        tot = sum(orc.solid_angle(p, *t) for t in tris) / (4 * math.pi)
        assert tot == pytest.approx(w, abs=1e-12)


# -------------------------------------------------------- Lagrange map --

REF = np.array([[a - 1, b - 1, c - 1] for c in range(3) for b in range(3) for a in range(3)], float)


def test_q2_partition_of_unity_and_affine(orc):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    b = rng.standard_normal(3)
    X = REF @ A.T + b
    for _ in range(20):
        xi = rng.uniform(-1.2, 1.2, 3)
        x, J = orc.q2_eval(X, xi)
        np.testing.assert_allclose(x, A @ xi + b, atol=1e-13)
        np.testing.assert_allclose(J, A, atol=1e-13)
    Xc = np.tile([0.3, -1.25, 7.0], (27, 1))
    x, J = orc.q2_eval(Xc, [0.3, -0.7, 0.1])
    np.testing.assert_allclose(x, [0.3, -1.25, 7.0], atol=1e-14)
    np.testing.assert_allclose(J, 0.0, atol=1e-14)


def test_q2_interpolates_nodes_and_derivative(orc):
    rng = np.random.default_rng(2)
    X = REF * 0.5 + 0.05 * rng.standard_normal((27, 3))
    for n in range(27):
        x, _ = orc.q2_eval(X, REF[n])
        np.testing.assert_allclose(x, X[n], atol=1e-15)
    xi = np.array([0.2, -0.4, 0.7])
    _, J = orc.q2_eval(X, xi)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        xp, _ = orc.q2_eval(X, xi + e)
        xm, _ = orc.q2_eval(X, xi - e)
        np.testing.assert_allclose((xp - xm) / (2 * h), J[:, j], atol=1e-9)


# ----------------------------------------------------------------- Newton --

def test_newton_affine_closed_form(orc):
    h, c = 0.25, np.array([0.3, -0.1, 1.2])
    X = c + 0.5 * h * REF
    rng = np.random.default_rng(3)
    for _ in range(20):
        xp = c + rng.uniform(-0.5 * h, 0.5 * h, 3)
        ok, xi, it = orc.newton(X, xp)
        assert ok
        assert it <= 3
        np.testing.assert_allclose(xi, (xp - c) / (0.5 * h), atol=1e-15)


def test_newton_self_donor_gauss_points(orc):
    rng = np.random.default_rng(4)
    X = 0.1 * REF + 0.006 * rng.standard_normal((27, 3))
    g = math.sqrt(0.6)
    for c in (-g, 0, g):
        for b in (-g, 0, g):
            for a in (-g, 0, g):
                xp, _ = orc.q2_eval(X, [a, b, c])
                ok, xi, _ = orc.newton(X, xp)
                assert ok
                np.testing.assert_allclose(xi, [a, b, c], atol=1e-12)


def test_newton_outside_point_not_contained(orc):
    X = 0.1 * REF
    ok, xi, _ = orc.newton(X, [0.1 * 1.2, 0.0, 0.0])
    assert not ok
    ok, xi, _ = orc.newton(X, [0.1 * 1.005, 0.0, 0.0])
    assert not ok and xi[0] == pytest.approx(1.005, abs=1e-12)


# --------------------------------------------------------------- neighbours --

def test_face_neighbors_structured(orc):
    from workloads import meshes as M
    g = M.background_grid((3, 4, 5), -1, 1, amp=0.0)
    nbr = orc.face_neighbors(g.conn)
    nx, ny, nz = 3, 4, 5
    for e in range(g.n_elem):
        i, j, k = e % nx, (e // nx) % ny, e // (nx * ny)
        exp = [e - 1 if i > 0 else -1, e + 1 if i < nx - 1 else -1,
               e - nx if j > 0 else -1, e + nx if j < ny - 1 else -1,
               e - nx * ny if k > 0 else -1, e + nx * ny if k < nz - 1 else -1]
        assert list(nbr[e]) == exp
