"""Pins of the oracle's artificial-boundary pieces (Sec. 2): AB faces from a
closed-form box cut and from a near-body grid's overset tags, flux points
in closed form on an undisplaced grid and shared between the two sides of
a face, interpolation weights that reproduce polynomials (no GPU)."""
import numpy as np

from workloads import meshes as M


def _cells(n, lo, hi):
    e = np.linspace(lo, hi, n + 1)
    return e[:-1], e[1:]


def _block_range(n, lo, hi, a, b):
    """Index ranges of the cells of an undisplaced n^3 grid meeting the
    closed box [a, b], per axis."""
    l, u = _cells(n, lo, hi)
    out = []
    for ax in range(3):
        idx = np.nonzero((u >= a[ax]) & (l <= b[ax]))[0]
        out.append((int(idx[0]), int(idx[-1])))
    return out


def test_ab_faces_box_closed_form(orc):
    """A box wall cuts a block of cells; the AB faces are the block's outer
    skin seen from the cells just outside it: 2(ab + bc + ca) faces, each
    named by the outside cell and its face towards the block."""
    n, lo, hi = 12, -1.2, 1.2
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = np.array([-0.41, -0.33, -0.27]), np.array([0.36, 0.52, 0.31])
    s = M.box_surface(2, a, b)
    ib = orc.cut(g, [s], [M.IDENTITY_POSE])
    (i0, i1), (j0, j1), (k0, k1) = _block_range(n, lo, hi, a, b)
    eid = lambda i, j, k: i + n * j + n * n * k
    want = []
    for j in range(j0, j1 + 1):
        for k in range(k0, k1 + 1):
            want += [6 * eid(i0 - 1, j, k) + 1, 6 * eid(i1 + 1, j, k) + 0]
    for i in range(i0, i1 + 1):
        for k in range(k0, k1 + 1):
            want += [6 * eid(i, j0 - 1, k) + 3, 6 * eid(i, j1 + 1, k) + 2]
        for j in range(j0, j1 + 1):
            want += [6 * eid(i, j, k0 - 1) + 5, 6 * eid(i, j, k1 + 1) + 4]
    A, B, Cn = i1 - i0 + 1, j1 - j0 + 1, k1 - k0 + 1
    got = orc.ab_faces(g, ib)
    assert got.size == 2 * (A * B + B * Cn + Cn * A)
    assert np.array_equal(got, np.sort(np.array(want)))


def test_ab_faces_overset_tags(orc):
    """A near-body grid with no hole: its AB faces are exactly its
    overset-tagged faces, one per face of the wall it wraps."""
    s = M.cube_sphere(4, R=0.5)
    sh = M.shell_grid(s, 3, r_out=1.0)
    ib = orc.cut(sh, [], [])
    got = orc.ab_faces(sh, ib)
    tags = np.asarray(sh.face_tags)
    want = np.nonzero(tags.reshape(-1) == orc.TAG_OVERSET)[0]
    assert np.array_equal(got, want) and got.size == s.conn.shape[0]


def test_ab_faces_pair_holes_with_kept_cells(orc):
    """Dimpled sphere on a displaced grid: every AB face without an overset
    tag joins a kept cell to a hole, and every (kept, hole) neighbour pair
    is named once."""
    g = M.background_grid(12, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(5, R=0.5, dimples=20, dimple_a=0.09, dimple_k=0.03)
    ib = orc.cut(g, [s], [M.pose_rz(0.3, (0.05, 0, 0))])
    nbr = orc.face_neighbors(g.conn)
    got = orc.ab_faces(g, ib, nbr)
    e, f = got // 6, got % 6
    assert np.all(ib[e] != orc.HOLE)
    assert np.all(ib[nbr[e, f]] == orc.HOLE)
    pairs = {(int(x), int(nbr[x, y])) for x, y in zip(e, f)}
    assert len(pairs) == got.size
    h = np.nonzero(ib == orc.HOLE)[0]
    expect = {(int(nbr[x, y]), int(x)) for x in h for y in range(6)
              if nbr[x, y] >= 0 and ib[nbr[x, y]] != orc.HOLE}
    assert pairs == expect and got.size > 0


def test_face_points_closed_form(orc):
    """Undisplaced grid: the flux points of face f of cell (i, j, k) lie on
    the cell's face plane at the Gauss points of its square."""
    n, lo, hi = 5, -1.0, 1.5
    h = (hi - lo) / n
    g = M.background_grid(n, lo, hi, amp=0.0)
    faces = np.arange(6 * g.n_elem)[::7]
    pts = orc.face_points(g, faces).reshape(-1, 9, 3)
    z = orc.GAUSS3
    for fid, P in zip(faces, pts):
        e, f = divmod(int(fid), 6)
        idx = [e % n, (e // n) % n, e // (n * n)]
        d = f // 2
        u, v = [k for k in range(3) if k != d]
        for q in range(9):
            a, b = q % 3, q // 3
            want = np.empty(3)
            want[d] = lo + (idx[d] + f % 2) * h
            want[u] = lo + (idx[u] + (1 + z[a]) / 2) * h
            want[v] = lo + (idx[v] + (1 + z[b]) / 2) * h
            assert np.abs(P[q] - want).max() <= 1e-14


def test_face_points_shared_between_sides(orc):
    """Displaced grid: the +xi (+eta, +zeta) face of a cell and the -xi
    (-eta, -zeta) face of its neighbour carry the same flux points in the
    same order."""
    g = M.background_grid(6, -1.0, 1.0, amp=0.05)
    nbr = orc.face_neighbors(g.conn)
    for f in (1, 3, 5):
        e = np.nonzero(nbr[:, f] >= 0)[0]
        q = nbr[e, f]
        assert np.all(nbr[q, f - 1] == e)
        P = orc.face_points(g, 6 * e + f)
        Q = orc.face_points(g, 6 * q + f - 1)
        assert np.abs(P - Q).max() <= 1e-14


def test_face_points_match_the_map_evaluator(orc):
    """The numpy map of the flux points against the C evaluator of
    eq. reftophys, on a curved shell, posed."""
    s = M.cube_sphere(3, R=0.5, dimples=6, dimple_a=0.1, dimple_k=0.02)
    sh = M.shell_grid(s, 2, r_out=1.0)
    pose = M.pose_rz(0.7, (0.2, -0.1, 0.3))
    rng = np.random.default_rng(5)
    faces = rng.choice(6 * sh.n_elem, 40, replace=False)
    P = orc.face_points(sh, faces, pose=pose).reshape(-1, 9, 3)
    R, t = pose[:9].reshape(3, 3), pose[9:]
    for fid, Pf in zip(faces, P):
        e, f = divmod(int(fid), 6)
        X = sh.nodes[sh.conn[e]]
        for q, xi in enumerate(orc.face_reference_points(f, orc.GAUSS3)):
            x, _ = orc.q2_eval(X, xi)
            assert np.abs(Pf[q] - (R @ x + t)).max() <= 1e-13


def test_interp_weights_reproduce_polynomials(orc):
    """Partition of unity, the Kronecker property at the nodes, exact
    reproduction of tensor polynomials of degree < m, NaN for orphans; for
    the 3-point Gauss nodes and the 5-point Gauss-Lobatto nodes."""
    rng = np.random.default_rng(11)
    lob5 = np.array([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0])
    for z in (orc.GAUSS3, lob5):
        m = z.size
        ref = rng.uniform(-1.0, 1.0, (50, 3))
        donor = np.arange(50)
        donor[7] = -1
        W = orc.interp_weights(donor, ref, z)
        assert W.shape == (50, m ** 3)
        assert np.all(np.isnan(W[7])) and not np.any(np.isnan(np.delete(W, 7, axis=0)))
        ok = donor >= 0
        assert np.abs(W[ok].sum(axis=1) - 1.0).max() <= 1e-13
        c = rng.normal(size=(m, m, m))
        node = np.array([(z[k % m], z[(k // m) % m], z[k // (m * m)]) for k in range(m ** 3)])
        qv = lambda p: sum(c[i, j, k] * p[..., 0] ** i * p[..., 1] ** j * p[..., 2] ** k
                           for i in range(m) for j in range(m) for k in range(m))
        assert np.abs(W[ok] @ qv(node) - qv(ref[ok])).max() <= 1e-11
        K = orc.interp_weights(np.zeros(m ** 3, dtype=np.int64), node, z)
        assert np.abs(K - np.eye(m ** 3)).max() <= 1e-14
