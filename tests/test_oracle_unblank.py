"""Pins of the oracle's unblank procedure (Alg. unblank): closed-form box
motions under the wall and overset rules, the degenerate cases, invariants
(no GPU)."""
import numpy as np

from workloads import meshes as M


def _cells(n, lo, hi):
    e = np.linspace(lo, hi, n + 1)
    return e[:-1], e[1:]


def _block(n, lo, hi, a, b, strict=False):
    """Cells of an undisplaced n^3 grid meeting the closed box [a, b]
    (strict: lying strictly inside it), as a boolean mask."""
    l, u = _cells(n, lo, hi)
    e = np.arange(n ** 3)
    idx = [e % n, (e // n) % n, e // n ** 2]
    m = np.ones(n ** 3, dtype=bool)
    for ax in range(3):
        ok = ((l > a[ax]) & (u < b[ax])) if strict else ((u >= a[ax]) & (l <= b[ax]))
        m &= ok[idx[ax]]
    return m


def _shift(p, d):
    q = p.copy()
    q[9:] += d
    return q


def test_unblank_wall_box_closed_form(orc):
    """A box wall moving along x: the new holes are the cells meeting the box
    at t or at t + dt; the cells to unblank are the previous holes outside
    both (three positions, closed form per axis)."""
    n, lo, hi = 14, -1.4, 1.4
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = np.array([-0.41, -0.33, -0.27]), np.array([0.36, 0.52, 0.31])
    s = M.box_surface(2, a, b)
    I = M.IDENTITY_POSE
    d_prev, d_t, d_tp = -0.23, 0.0, 0.26
    prev = orc.cut(g, [s], [_shift(I, [d_prev, 0, 0])])
    ib, ub = orc.unblank(g, [s], [_shift(I, [d_t, 0, 0])], [_shift(I, [d_tp, 0, 0])], prev)
    h_prev = _block(n, lo, hi, a + [d_prev, 0, 0], b + [d_prev, 0, 0])
    h_t = _block(n, lo, hi, a + [d_t, 0, 0], b + [d_t, 0, 0])
    h_tp = _block(n, lo, hi, a + [d_tp, 0, 0], b + [d_tp, 0, 0])
    assert np.array_equal(prev == orc.HOLE, h_prev)
    assert np.array_equal(ib == orc.HOLE, h_t | h_tp)
    assert np.array_equal(ub, np.nonzero(h_prev & ~(h_t | h_tp))[0])
    assert ub.size > 0
    # the new fringe is the face layer around the union of the two blocks
    nbr = orc.face_neighbors(g.conn)
    assert np.array_equal(ib, orc.mark_fringe(h_t | h_tp, nbr))


def test_unblank_overset_box_closed_form(orc):
    """Overset rule: a hole only where both cuts agree (cells strictly inside
    the box at t and at t + dt); the previous holes outside that set are
    unblanked."""
    n, lo, hi = 12, -1.2, 1.2
    g = M.background_grid(n, lo, hi, amp=0.0)
    a, b = np.array([-0.63, -0.58, -0.49]), np.array([0.55, 0.61, 0.47])
    s = M.box_surface(2, a, b)
    I = M.IDENTITY_POSE
    moves = ([0.0, -0.17, 0.0], [0.0, 0.0, 0.0], [0.0, 0.21, 0.0])
    prev_h = _block(n, lo, hi, a + moves[0], b + moves[0], strict=True)
    prev = np.where(prev_h, orc.HOLE, orc.FIELD).astype(np.int8)
    ib, ub = orc.unblank(g, [s], [_shift(I, moves[1])], [_shift(I, moves[2])], prev, kind=orc.SURF_OVERSET)
    h_t = _block(n, lo, hi, a + moves[1], b + moves[1], strict=True)
    h_tp = _block(n, lo, hi, a + moves[2], b + moves[2], strict=True)
    assert np.array_equal(ib == orc.HOLE, h_t & h_tp)
    assert np.array_equal(ub, np.nonzero(prev_h & ~(h_t & h_tp))[0])
    assert ub.size > 0


def test_unblank_degenerate_cases(orc):
    """Same pose at t and t + dt: the blanking is the plain cut; a body at
    rest (previous blanking = current) unblanks nothing; an empty previous
    blanking unblanks nothing."""
    g = M.background_grid(10, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(4, R=0.45, dimples=10, dimple_a=0.08, dimple_k=0.02)
    p = M.pose_rz(0.3, (0.05, -0.02, 0.04))
    cut = orc.cut(g, [s], [p])
    for kind in (orc.SURF_WALL, orc.SURF_OVERSET):
        ref = orc.cut(g, [s], [p], kinds=[kind])
        ib, ub = orc.unblank(g, [s], [p], [p], ref, kind=kind)
        assert np.array_equal(ib, ref) and ub.size == 0
    ib, ub = orc.unblank(g, [s], [p], [p], np.ones(g.n_elem, dtype=np.int8))
    assert np.array_equal(ib, cut) and ub.size == 0


def test_unblank_invariants(orc):
    """Spinning dimpled sphere, wall rule: the new holes contain both cuts'
    holes, no unblanked cell is a hole, every unblanked cell was a hole."""
    g = M.background_grid(12, -1.2, 1.2, amp=0.03)
    s = M.cube_sphere(5, R=0.5, dimples=20, dimple_a=0.09, dimple_k=0.03, axes=(1.0, 0.8, 0.6))
    poses = [M.pose_rz(0.35 * k, (0.04 * k, 0, 0)) for k in range(3)]
    prev = orc.cut(g, [s], [poses[0]])
    ib, ub = orc.unblank(g, [s], [poses[1]], [poses[2]], prev)
    h = ib == orc.HOLE
    assert np.all(h[orc.cut(g, [s], [poses[1]]) == orc.HOLE])
    assert np.all(h[orc.cut(g, [s], [poses[2]]) == orc.HOLE])
    assert not np.any(h[ub])
    assert np.all(prev[ub] == orc.HOLE)
    assert ub.size > 0 and np.all(np.diff(ub) > 0)
