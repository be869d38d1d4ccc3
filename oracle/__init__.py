"""Plain FP64 CPU oracle for the overset direct cut and donor search.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_1711_07663_amd``; the C source in
``oracle.c`` is compiled by :func:`build` with gcc.

Functions follow the paper (Crabill, Witherden & Jameson, arXiv:1711.07663):

* :func:`cut` -- Sec. 4.2 (parallel direct cut), the per-surface status, the
  union of holes over cutting surfaces and the artificial-boundary (fringe)
  layer of Sec. 4.2's last paragraphs.
* :func:`unblank` -- Sec. 3, Alg. unblank: the blanking of a moving grid's
  time step from the cuts at t and t + dt, and the cells to unblank.
* :func:`fringe_points` -- receptor points: a 3x3x3 Gauss-Legendre tensor per
  fringe element mapped by eq. reftophys.
* :func:`donor_search` -- Sec. 4.3, Newton inversion of eq. reftophys with
  eq. ref-update / eq. Jac, at most 10 iterations, clamped near [-1, 1].
* :func:`cut_heuristic` -- the paper's own filtered cut (Sec. 4.2, Alg. cp0,
  bboxdix, cp1, cp2): approximate distances, the nearest N_F^1 faces, a
  linear first pass keeping N_F^2 of them, the lattice second pass at the
  nearest corner, the nearest pair's normal side.
* :func:`ab_faces`, :func:`face_points`, :func:`interp_weights` -- the
  artificial-boundary (AB) method of Sec. 2: the faces between a hole and a
  kept element (and overset-tagged faces), the flux points on them (the
  receptor points of the AB method), and the Lagrange weights that query a
  donor's solution polynomial at a receptor's reference location.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HOLE, FIELD, FRINGE = 0, 1, -1
SURF_WALL, SURF_OVERSET = 0, 1
TAG_OVERSET = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c to load (the sanitizer test's)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so (gcc, FP64, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(src):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path):
    """Compile oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    into path (a checking build for tests; loaded through ORACLE_LIB with the
    ASan runtime preloaded)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", src,
           "-o", path, "-lm"]
    subprocess.run(cmd, check=True)
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp, ip, i8p, i64p = (C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int8),
                             C.POINTER(C.c_int64))
        L.orc_tri_tri.restype = C.c_double
        L.orc_tri_tri.argtypes = [dp, dp, dp, dp]
        L.orc_solid_angle.restype = C.c_double
        L.orc_solid_angle.argtypes = [dp, dp, dp, dp]
        L.orc_q2_eval.restype = None
        L.orc_q2_eval.argtypes = [dp, dp, dp, dp]
        L.orc_newton.restype = C.c_int
        L.orc_newton.argtypes = [dp, dp, C.c_int, dp, C.POINTER(C.c_int)]
        L.orc_face_neighbors.restype = C.c_int
        L.orc_face_neighbors.argtypes = [ip, C.c_int64, ip]
        L.orc_element_winding.restype = C.c_double
        L.orc_element_winding.argtypes = [dp, ip, C.c_int64, dp]
        L.orc_element_tris.restype = None
        L.orc_element_tris.argtypes = [dp, ip, C.c_int64, dp]
        L.orc_cut_surface.restype = C.c_int
        L.orc_cut_surface.argtypes = [dp, ip, C.c_int64, i64p, C.c_int64, dp, C.c_int64, ip, C.c_int64,
                                      dp, C.c_int, C.c_int, C.c_int, i8p, i8p, dp, i8p, dp, i8p]
        L.orc_cut_heuristic.restype = C.c_int
        L.orc_cut_heuristic.argtypes = [dp, ip, C.c_int64, dp, C.c_int64, ip, C.c_int64, dp, C.c_int, C.c_int,
                                        C.c_int, C.c_int, i8p, i8p]
        L.orc_hx_obb.restype = None
        L.orc_hx_obb.argtypes = [dp, dp]
        L.orc_hx_bbox_dist.restype = C.c_double
        L.orc_hx_bbox_dist.argtypes = [dp, dp]
        L.orc_hx_lists.restype = C.c_int
        L.orc_hx_lists.argtypes = [dp, dp, ip, C.c_int64, dp, C.c_int, C.c_int, i64p, dp, i64p, dp, ip]
        L.orc_fringe_points.restype = C.c_int
        L.orc_fringe_points.argtypes = [dp, ip, i64p, C.c_int64, dp, dp]
        L.orc_donor_search.restype = C.c_int
        L.orc_donor_search.argtypes = [dp, ip, C.c_int64, dp, dp, C.c_int64, C.c_int, C.c_int, C.c_int,
                                       ip, dp, ip, ip]
        _lib = L
    return _lib


def _p(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


IDENTITY = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=np.float64)


# ---------------------------------------------------------------------------
# primitives (exposed for the pin tests)
# ---------------------------------------------------------------------------

def tri_tri(A, B):
    """Distance between triangles A, B (3x3 arrays) and the closest points."""
    A = _f64(A).reshape(9)
    B = _f64(B).reshape(9)
    pa = np.zeros(3)
    pb = np.zeros(3)
    d = lib().orc_tri_tri(_p(A, C.c_double), _p(B, C.c_double), _p(pa, C.c_double), _p(pb, C.c_double))
    return d, pa, pb


def solid_angle(p, a, b, c):
    p, a, b, c = (_f64(v).reshape(3) for v in (p, a, b, c))
    return lib().orc_solid_angle(*(_p(v, C.c_double) for v in (p, a, b, c)))


def q2_eval(X, xi):
    """x(xi) and J = dx/dxi of a 27-node element (X: 27x3)."""
    X = _f64(X).reshape(81)
    xi = _f64(xi).reshape(3)
    x = np.zeros(3)
    J = np.zeros(9)
    lib().orc_q2_eval(_p(X, C.c_double), _p(xi, C.c_double), _p(x, C.c_double), _p(J, C.c_double))
    return x, J.reshape(3, 3)


def newton(X, xp, maxit=10):
    X = _f64(X).reshape(81)
    xp = _f64(xp).reshape(3)
    xi = np.zeros(3)
    it = C.c_int(0)
    ok = lib().orc_newton(_p(X, C.c_double), _p(xp, C.c_double), int(maxit), _p(xi, C.c_double), C.byref(it))
    return bool(ok), xi, it.value


def element_tris(nodes, conn, e):
    nodes = _f64(nodes)
    conn = _i32(conn)
    out = np.zeros(48 * 9)
    lib().orc_element_tris(_p(nodes, C.c_double), _p(conn, C.c_int32), int(e), _p(out, C.c_double))
    return out.reshape(48, 3, 3)


def element_winding(nodes, conn, e, p):
    nodes = _f64(nodes)
    conn = _i32(conn)
    p = _f64(p).reshape(3)
    return lib().orc_element_winding(_p(nodes, C.c_double), _p(conn, C.c_int32), int(e), _p(p, C.c_double))


def face_neighbors(conn):
    conn = _i32(conn)
    n = conn.shape[0]
    nbr = np.empty((n, 6), dtype=np.int32)
    rc = lib().orc_face_neighbors(_p(conn, C.c_int32), n, _p(nbr, C.c_int32))
    if rc != 0:
        raise MemoryError("orc_face_neighbors")
    return nbr


# ---------------------------------------------------------------------------
# cut
# ---------------------------------------------------------------------------

def cut_surface(grid, surf, pose=IDENTITY, kind=SURF_WALL, sel=None, brute=False, threads=0,
                diagnostics=False):
    """Per-surface status of the selected elements (0 hole / 1 field).

    With ``diagnostics`` also returns hit flags, the global nearest distance,
    the nearest-face side (+1 outside / -1 inside) from the element-surface
    nearest triangle pair, the winding number at each element's first node
    and the nearest-face side of that node (``psign``).  ``diagnostics`` may
    be "point" to skip the element-pair search."""
    gn = _f64(grid.nodes)
    gc = _i32(grid.conn)
    sn = _f64(surf.nodes)
    sc = _i32(surf.conn)
    pose = _f64(pose)
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
    n = gc.shape[0] if sel is None else sel.shape[0]
    status = np.empty(n, dtype=np.int8)
    hit = np.empty(n, dtype=np.int8)
    pair = diagnostics is True
    dstar = np.empty(n) if pair else None
    nsign = np.empty(n, dtype=np.int8) if pair else None
    wind = np.empty(n) if diagnostics else None
    psign = np.empty(n, dtype=np.int8) if diagnostics else None
    lib().orc_cut_surface(_p(gn, C.c_double), _p(gc, C.c_int32), gc.shape[0], _p(sel, C.c_int64),
                          0 if sel is None else sel.shape[0], _p(sn, C.c_double), sn.shape[0],
                          _p(sc, C.c_int32), sc.shape[0], _p(pose, C.c_double), int(kind), int(bool(brute)),
                          int(threads), _p(status, C.c_int8), _p(hit, C.c_int8), _p(dstar, C.c_double),
                          _p(nsign, C.c_int8), _p(wind, C.c_double), _p(psign, C.c_int8))
    if diagnostics:
        return dict(status=status, hit=hit, dstar=dstar, nsign=nsign, wind=wind, psign=psign)
    return status


def mark_fringe(hole, nbr, face_tags=None):
    """iblank from a hole mask: field elements that share a face with a hole,
    or carry an overset-tagged face, become fringe (-1)."""
    hole = np.asarray(hole, dtype=bool)
    ib = np.where(hole, HOLE, FIELD).astype(np.int8)
    nb_hole = np.zeros(hole.shape[0], dtype=bool)
    for f in range(6):
        nb = nbr[:, f]
        ok = nb >= 0
        nb_hole[ok] |= hole[nb[ok]]
    fr = (~hole) & nb_hole
    if face_tags is not None:
        fr |= (~hole) & (np.asarray(face_tags) == TAG_OVERSET).any(axis=1)
    ib[fr] = FRINGE
    return ib


def cut(grid, surfaces, poses, kinds=None, nbr=None, brute=False, threads=0):
    """iblank of ``grid`` cut by several posed surfaces: union of holes over
    the surfaces, then one fringe layer (hole 0, field 1, fringe -1)."""
    if kinds is None:
        kinds = [SURF_WALL] * len(surfaces)
    hole = np.zeros(grid.conn.shape[0], dtype=bool)
    for s, p, k in zip(surfaces, poses, kinds):
        hole |= cut_surface(grid, s, p, k, brute=brute, threads=threads) == 0
    if nbr is None:
        nbr = face_neighbors(grid.conn)
    return mark_fringe(hole, nbr, grid.face_tags)


def hole_mask(grid, surfaces, poses, kind=SURF_WALL, threads=0):
    """Union over the surfaces of their holes in ``grid`` (Sec. 4.2)."""
    hole = np.zeros(grid.conn.shape[0], dtype=bool)
    for s, p in zip(surfaces, poses):
        hole |= cut_surface(grid, s, p, kind, threads=threads) == 0
    return hole


def unblank(grid, surfaces, poses_t, poses_tp, prev_iblank, kind=SURF_WALL, nbr=None, threads=0):
    """Blanking of one time step with unblanking (Alg. unblank, steps 3-8),
    for a grid cut by surfaces of one kind.

    I_t and I_{t+} are the hole sets of the cuts at the poses of time t and
    t + dt.  A grid cut by solid walls takes the holes of either
    (a cell that becomes a hole at t + dt is a hole now); a grid cut by
    overset boundaries keeps a hole only where both cuts agree (cells are
    not blanked before they are known not to be needed, and are unblanked
    before they are needed).  The cells to unblank are the holes of the
    previous blanking (``prev_iblank``, I_{t-}) that are not holes of the
    new one.  Returns the new iblank (one fringe layer around its holes,
    overset-tagged faces fringe) and the ascending ids of the cells to
    unblank."""
    h_t = hole_mask(grid, surfaces, poses_t, kind, threads)
    h_tp = hole_mask(grid, surfaces, poses_tp, kind, threads)
    hole = (h_t | h_tp) if kind == SURF_WALL else (h_t & h_tp)
    if nbr is None:
        nbr = face_neighbors(grid.conn)
    ib = mark_fringe(hole, nbr, grid.face_tags)
    ub = np.nonzero((np.asarray(prev_iblank) == HOLE) & ~hole)[0].astype(np.int64)
    return ib, ub


def fringe_elements(iblank):
    return np.nonzero(np.asarray(iblank) == FRINGE)[0].astype(np.int64)


def fringe_points(grid, elems, pose=IDENTITY):
    """27 Gauss points per element (order a + 3b + 9c), mapped and posed."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    gn = _f64(grid.nodes)
    gc = _i32(grid.conn)
    pose = _f64(pose)
    pts = np.empty((elems.shape[0] * 27, 3))
    lib().orc_fringe_points(_p(gn, C.c_double), _p(gc, C.c_int32), _p(elems, C.c_int64), elems.shape[0],
                            _p(pose, C.c_double), _p(pts, C.c_double))
    return pts


def donor_search(grid, pts, pose=IDENTITY, brute=False, maxit=10, threads=0):
    """Donor element (-1 = orphan) and reference coordinates of world points."""
    gn = _f64(grid.nodes)
    gc = _i32(grid.conn)
    pose = _f64(pose)
    pts = _f64(pts).reshape(-1, 3)
    n = pts.shape[0]
    donor = np.empty(n, dtype=np.int32)
    xi = np.empty((n, 3))
    iters = np.empty(n, dtype=np.int32)
    ncand = np.empty(n, dtype=np.int32)
    lib().orc_donor_search(_p(gn, C.c_double), _p(gc, C.c_int32), gc.shape[0], _p(pose, C.c_double),
                           _p(pts, C.c_double), n, int(bool(brute)), int(maxit), int(threads),
                           _p(donor, C.c_int32), _p(xi, C.c_double), _p(iters, C.c_int32),
                           _p(ncand, C.c_int32))
    return donor, xi, dict(iters=iters, n_cand=ncand)


# ---------------------------------------------------------------------------
# artificial-boundary faces, flux points, interpolation weights (Sec. 2)
# ---------------------------------------------------------------------------

def ab_faces(grid, iblank, nbr=None):
    """Artificial-boundary faces (Sec. 2, step 1; Sec. 4.2, last paragraph):
    a face with a hole on one side and a kept (field or fringe) element on
    the other, plus the overset-tagged faces of kept elements (the outer
    boundary of a near-body grid, where the AB method exchanges data).
    Each face is named from its kept side, id = 6 e + f (f in the order
    -xi, +xi, -eta, +eta, -zeta, +zeta); ids ascending."""
    ib = np.asarray(iblank)
    if nbr is None:
        nbr = face_neighbors(grid.conn)
    kept = ib != HOLE
    out = []
    for f in range(6):
        nb = nbr[:, f]
        ab = kept & (nb >= 0)
        ab[ab] = ib[nb[ab]] == HOLE
        if grid.face_tags is not None:
            ab |= kept & (np.asarray(grid.face_tags)[:, f] == TAG_OVERSET)
        out.append(6 * np.nonzero(ab)[0].astype(np.int64) + f)
    return np.sort(np.concatenate(out))


def lagrange_1d(nodes1d, s):
    """Lagrange basis through the 1-D nodes, at the values s: (len(s), m)."""
    z = np.asarray(nodes1d, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64).reshape(-1)
    L = np.ones((s.size, z.size))
    for i in range(z.size):
        for j in range(z.size):
            if j != i:
                L[:, i] *= (s - z[j]) / (z[i] - z[j])
    return L


def q2_map_points(grid, elems, xi, pose=IDENTITY):
    """x(xi) of eq. reftophys for element elems[k] at reference point xi[k]
    (quadratic Lagrange basis on the equispaced nodes -1, 0, 1, node order
    a + 3b + 9c), then posed: R x + t."""
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    xi = np.asarray(xi, dtype=np.float64).reshape(-1, 3)
    eq = np.array([-1.0, 0.0, 1.0])
    La, Lb, Lc = (lagrange_1d(eq, xi[:, d]) for d in range(3))
    W = (La[:, None, None, :] * Lb[:, None, :, None] * Lc[:, :, None, None]).reshape(-1, 27)
    X = np.asarray(grid.nodes, dtype=np.float64)[np.asarray(grid.conn)[elems]]   # (n, 27, 3)
    x = np.einsum("nk,nkd->nd", W, X)
    pose = np.asarray(pose, dtype=np.float64)
    return x @ pose[:9].reshape(3, 3).T + pose[9:]


def face_reference_points(f, nodes1d):
    """Reference coordinates of the m x m flux points of local face f: the
    face's own axis at -1 (f even) or +1 (f odd); the two other axes, in
    increasing axis order, take nodes1d[a] and nodes1d[b], point a + m b."""
    z = np.asarray(nodes1d, dtype=np.float64)
    m = z.size
    d = f // 2
    u, v = [k for k in range(3) if k != d]
    out = np.empty((m * m, 3))
    out[:, d] = -1.0 if f % 2 == 0 else 1.0
    out[:, u] = np.tile(z, m)
    out[:, v] = np.repeat(z, m)
    return out


GAUSS3 = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])


def face_points(grid, faces, nodes1d=GAUSS3, pose=IDENTITY):
    """Flux points of the faces (ids 6 e + f): m x m points per face, order
    of face_reference_points, mapped by eq. reftophys and posed."""
    faces = np.asarray(faces, dtype=np.int64).reshape(-1)
    m = len(nodes1d)
    if faces.size == 0:
        return np.zeros((0, 3))
    refs = np.stack([face_reference_points(f, nodes1d) for f in range(6)])   # (6, m*m, 3)
    e = np.repeat(faces // 6, m * m)
    xi = refs[faces % 6].reshape(-1, 3)
    return q2_map_points(grid, e, xi, pose)


def interp_weights(donor, ref, nodes1d=GAUSS3):
    """Interpolation weights of the donor's nodal solution basis at each
    receptor's reference location (Sec. 2, step 3): the tensor Lagrange
    basis through nodes1d on each axis, weight a + m b + m^2 c =
    l_a(xi) l_b(eta) l_c(zeta).  Orphans (donor < 0) get NaN."""
    donor = np.asarray(donor).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    m = len(nodes1d)
    La, Lb, Lc = (lagrange_1d(nodes1d, ref[:, d]) for d in range(3))
    W = (La[:, None, None, :] * Lb[:, None, :, None] * Lc[:, :, None, None]).reshape(-1, m ** 3)
    W[donor < 0] = np.nan
    return W


# ---------------------------------------------------------------------------
# the paper's filtered cut (Sec. 4.2; Alg. cp0, bboxdix, cp1, cp2)
# ---------------------------------------------------------------------------

def hx_obb(X):
    """Element OBB of Alg. cp0 from the corner nodes of X (27 x 3): centroid,
    axes (rows: eigenvectors of the corner covariance), extents (lo3 hi3)."""
    X = _f64(X).reshape(81)
    o = np.zeros(18)
    lib().orc_hx_obb(_p(X, C.c_double), _p(o, C.c_double))
    return o[:3], o[3:12].reshape(3, 3), o[12:]


def hx_bbox_dist(b1, b2):
    """Alg. bboxdix between two 6-vector boxes (lo3 hi3)."""
    b1, b2 = _f64(b1).reshape(6), _f64(b2).reshape(6)
    return lib().orc_hx_bbox_dist(_p(b1, C.c_double), _p(b2, C.c_double))


def hx_lists(X, surf, pose=IDENTITY, nf1=16, nf2=4):
    """The filtered cut's kept lists for one element X (27 x 3): the nf1
    faces of smallest approximate distance (Alg. cp0) with their distances,
    then the nf2 of those of smallest first-pass distance (Alg. cp1) with
    their distances and kept corners."""
    X = _f64(X).reshape(81)
    sn, sc = _f64(surf.nodes), _i32(surf.conn)
    pose = _f64(pose)
    l1, d1 = np.empty(nf1, dtype=np.int64), np.empty(nf1)
    l2, d2, c2 = np.empty(nf2, dtype=np.int64), np.empty(nf2), np.empty(nf2, dtype=np.int32)
    rc = lib().orc_hx_lists(_p(X, C.c_double), _p(sn, C.c_double), _p(sc, C.c_int32), sc.shape[0],
                            _p(pose, C.c_double), int(nf1), int(nf2), _p(l1, C.c_int64), _p(d1, C.c_double),
                            _p(l2, C.c_int64), _p(d2, C.c_double), _p(c2, C.c_int32))
    if rc != 0:
        raise ValueError("orc_hx_lists: need 1 <= nf2 <= nf1 <= faces")
    return l1, d1, l2, d2, c2


def cut_surface_heuristic(grid, surf, pose=IDENTITY, kind=SURF_WALL, nf1=16, nf2=4, threads=0):
    """Per element status (0 hole, 1 field) and hit flag of the filtered cut."""
    gn, gc = _f64(grid.nodes), _i32(grid.conn)
    sn, sc = _f64(surf.nodes), _i32(surf.conn)
    pose = _f64(pose)
    n = gc.shape[0]
    st = np.empty(n, dtype=np.int8)
    hit = np.empty(n, dtype=np.int8)
    rc = lib().orc_cut_heuristic(_p(gn, C.c_double), _p(gc, C.c_int32), n, _p(sn, C.c_double), sn.shape[0],
                                 _p(sc, C.c_int32), sc.shape[0], _p(pose, C.c_double), int(kind), int(nf1), int(nf2),
                                 int(threads), _p(st, C.c_int8), _p(hit, C.c_int8))
    if rc != 0:
        raise ValueError("orc_cut_heuristic: nf1 and nf2 must be >= 1")
    return st, hit


def cut_heuristic(grid, surfaces, poses, kinds=None, nf1=16, nf2=4, nbr=None, threads=0):
    """iblank of the filtered cut: union of holes over the surfaces, then one
    fringe layer (as :func:`cut`)."""
    if kinds is None:
        kinds = [SURF_WALL] * len(surfaces)
    hole = np.zeros(grid.conn.shape[0], dtype=bool)
    for s, p, k in zip(surfaces, poses, kinds):
        hole |= cut_surface_heuristic(grid, s, p, k, nf1, nf2, threads)[0] == 0
    if nbr is None:
        nbr = face_neighbors(grid.conn)
    return mark_fringe(hole, nbr, grid.face_tags)


# ---------------------------------------------------------------------------
# refined (curved-face) cut
# ---------------------------------------------------------------------------
#
# The paper cuts with the node-lattice triangulation of every curved face
# (Sec. 4.2, Fig. quadsplit) and notes the linearisation error.  The refined
# cut of level k applies the same exact predicate to the curved geometry
# restricted to a finer lattice: every quadratic surface face is split into
# k x k quadratic sub-faces and every element into k^3 quadratic
# sub-elements, each the exact restriction of the isoparametric map
# (eq. reftophys) to a sub-square / sub-cube of the reference domain, so
# their 9 / 27 nodes are the map evaluated on the sub-lattice.  An element is
# a hole when any of its sub-elements is one (a closed surface that meets
# the element meets one of its pieces, and one that does not lies on the side
# of the element's first node, which is its first sub-element's first node).
# Level 1 is the lattice cut; the triangulations of level k lie within
# (M_uu + M_uv + M_vv) / k^2 of the curved faces (refinement_bound), so the
# predicate converges to the one on the curved faces.

class _Mesh:
    """Plain container of a grid (nodes, conn, face_tags) or a surface
    (nodes, conn) for the refined cut."""

    def __init__(self, nodes, conn, face_tags=None):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.face_tags = face_tags

    @property
    def n_elem(self):
        return int(self.conn.shape[0])

    @property
    def n_face(self):
        return int(self.conn.shape[0])


def _lag2(s):
    """Equispaced quadratic Lagrange values on the nodes -1, 0, 1 (eq.
    reftophys with K = 2), shape (..., 3)."""
    s = np.asarray(s, dtype=np.float64)
    return np.stack([0.5 * s * (s - 1.0), 1.0 - s * s, 0.5 * s * (s + 1.0)], axis=-1)


def _sub_params(k):
    """Reference coordinates of the level-k node lattice, -1 + I / k."""
    return -1.0 + np.arange(2 * k + 1, dtype=np.float64) / k


def refine_surface(surf, k):
    """The k x k quadratic sub-faces of every face of a surface of 9-node
    quads (node order a + 3b), as a surface of n_face k^2 faces.  Points on a
    face's boundary are evaluated from that edge's three nodes taken from the
    end with the lower node id, so faces sharing an edge share its refined
    points bit for bit (the refined surface stays watertight)."""
    if k == 1:
        return surf
    X = np.asarray(surf.nodes, dtype=np.float64)
    conn = np.asarray(surf.conn)
    N = 2 * k
    t = _sub_params(k)
    L = _lag2(t)                                      # (N+1, 3)
    nf = conn.shape[0]
    P = X[conn].reshape(nf, 3, 3, 3)                  # [f, b, a, xyz]  (node a + 3b)
    # interior: x(u_I, v_J) = sum_ab X_ab l_a(u_I) l_b(v_J)
    G = np.einsum("fbax,ia,jb->fijx", P, L, L)        # (nf, N+1, N+1, 3) indexed [I (u), J (v)]
    # edges, canonically: nodes (n0, n1, n2) along the edge; parameter from
    # the lower-id end
    def edge(ids, params_up):
        n0, n1, n2 = ids
        flip = n0 > n2
        s = np.where(flip[:, None], -params_up[None, :], params_up[None, :])
        lo = np.where(flip, n2, n0)
        hi = np.where(flip, n0, n2)
        l = _lag2(s)                                  # (nf, N+1, 3)
        return (X[lo][:, None, :] * l[:, :, 0:1] + X[n1][:, None, :] * l[:, :, 1:2]) + X[hi][:, None, :] * l[:, :, 2:3]
    G[:, :, 0, :] = edge((conn[:, 0], conn[:, 1], conn[:, 2]), t)          # v = -1, a = 0..2
    G[:, :, N, :] = edge((conn[:, 6], conn[:, 7], conn[:, 8]), t)          # v = +1
    G[:, 0, :, :] = edge((conn[:, 0], conn[:, 3], conn[:, 6]), t)          # u = -1, b = 0..2
    G[:, N, :, :] = edge((conn[:, 2], conn[:, 5], conn[:, 8]), t)          # u = +1
    nodes = []
    for bj in range(k):
        for bi in range(k):
            sub = G[:, 2 * bi:2 * bi + 3, 2 * bj:2 * bj + 3, :]            # [f, a, b]
            nodes.append(np.transpose(sub, (0, 2, 1, 3)).reshape(nf, 9, 3))  # node a + 3b
    nodes = np.stack(nodes, axis=1).reshape(nf * k * k, 9, 3)
    return _Mesh(nodes.reshape(-1, 3), np.arange(nf * k * k * 9, dtype=np.int32).reshape(-1, 9))


def refine_elements(grid, elems, k):
    """The k^3 quadratic sub-elements of each listed element (27 nodes
    a + 3b + 9c each, the element's map on a sub-cube), as a grid of
    len(elems) k^3 elements, element-major then sub-element (i + k j + k^2 l)."""
    X = np.asarray(grid.nodes, dtype=np.float64)[np.asarray(grid.conn)[np.asarray(elems)]]   # (n, 27, 3)
    n = X.shape[0]
    L = _lag2(_sub_params(k))
    Xc = X.reshape(n, 3, 3, 3, 3)                     # [e, c, b, a, xyz]
    G = np.einsum("ecbax,ia,jb,lc->eijlx", Xc, L, L, L)   # (n, N+1, N+1, N+1, 3) [I, J, L]
    subs = []
    for bl in range(k):
        for bj in range(k):
            for bi in range(k):
                s = G[:, 2 * bi:2 * bi + 3, 2 * bj:2 * bj + 3, 2 * bl:2 * bl + 3, :]   # [e, a, b, c]
                subs.append(np.transpose(s, (0, 3, 2, 1, 4)).reshape(n, 27, 3))       # a + 3b + 9c
    nodes = np.stack(subs, axis=1).reshape(n * k ** 3 * 27, 3)
    return _Mesh(nodes, np.arange(n * k ** 3 * 27, dtype=np.int32).reshape(-1, 27))


def _control_boxes(grid, elems):
    """Boxes of the Bernstein control nets of the listed elements (they hold
    the curved elements: convex-hull property)."""
    X = np.asarray(grid.nodes, dtype=np.float64)[np.asarray(grid.conn)[np.asarray(elems)]]
    B = X.reshape(-1, 3, 3, 3, 3).copy()              # [e, c, b, a, xyz]
    for ax in (3, 2, 1):
        idx = [slice(None)] * 5
        mid, lo_, hi_ = list(idx), list(idx), list(idx)
        mid[ax], lo_[ax], hi_[ax] = 1, 0, 2
        B[tuple(mid)] = 2.0 * B[tuple(mid)] - 0.5 * (B[tuple(lo_)] + B[tuple(hi_)])
    B = B.reshape(-1, 27, 3)
    return B.min(axis=1), B.max(axis=1)


def cut_surface_refined(grid, surf, k, pose=IDENTITY, kind=SURF_WALL, threads=0, pad=1e-4, sub_status=False):
    """Per-surface status (0 hole / 1 field) of every element of grid under
    the refined cut of level k.  Elements whose control-net box stays farther
    than pad from the posed refined surface's box are field (their curved
    extent is away from the surface, their first node outside it)."""
    sv = refine_surface(surf, k)
    R = np.asarray(pose[:9], dtype=np.float64).reshape(3, 3)
    Y = sv.nodes @ R.T + np.asarray(pose[9:12], dtype=np.float64)
    slo, shi = Y.min(axis=0) - pad, Y.max(axis=0) + pad
    n = grid.conn.shape[0]
    status = np.ones(n, dtype=np.int8)
    band = []
    for s0 in range(0, n, 1 << 16):
        ids = np.arange(s0, min(n, s0 + (1 << 16)))
        lo, hi = _control_boxes(grid, ids)
        band.append(ids[np.all(hi >= slo, axis=1) & np.all(lo <= shi, axis=1)])
    band = np.concatenate(band)
    if band.size == 0:
        return (status, band, np.zeros(0, dtype=np.int8)) if sub_status else status
    sub = refine_elements(grid, band, k)
    st = cut_surface(sub, sv, pose, kind, threads=threads)
    hole = (st.reshape(band.size, k ** 3) == 0).any(axis=1)
    status[band[hole]] = 0
    return (status, band, st) if sub_status else status


def cut_refined(grid, surfaces, poses, k, kinds=None, nbr=None, threads=0):
    """iblank of grid under the refined cut of level k: union of holes over
    the surfaces, then one fringe layer."""
    if kinds is None:
        kinds = [SURF_WALL] * len(surfaces)
    hole = np.zeros(grid.conn.shape[0], dtype=bool)
    for s, p, kd in zip(surfaces, poses, kinds):
        hole |= cut_surface_refined(grid, s, k, p, kd, threads=threads) == 0
    if nbr is None:
        nbr = face_neighbors(grid.conn)
    return mark_fringe(hole, nbr, grid.face_tags)


def refinement_bound(nodes9, k):
    """Bound on the distance between a quadratic patch (9 nodes, a + 3b, on
    [-1,1]^2) and its level-k lattice triangulation (2k x 2k sub-quads of
    parameter side h = 1/k, two triangles each): on a triangle, linear
    interpolation misses f by at most M R^2 / 2 with R the circumradius
    (h / sqrt 2) and M a bound on |D^2 x [d, d]| for unit d, here
    |x_uu| + |x_uv| + |x_vv| maximised over the patch: x_uu and x_vv are
    quadratics in one variable (bounded by their Bernstein control points),
    x_uv is bilinear (bounded at the corners).  Returns M h^2 / 4."""
    P = np.asarray(nodes9, dtype=np.float64).reshape(3, 3, 3)     # [b, a, xyz]
    d2 = np.array([1.0, -2.0, 1.0])
    def bern_max(c):                                               # c: (3, 3) values at -1, 0, 1
        b = np.stack([c[0], 2.0 * c[1] - 0.5 * (c[0] + c[2]), c[2]])
        return np.linalg.norm(b, axis=1).max()
    xuu = np.einsum("bax,a->bx", P, d2)                            # x_uu at v = -1, 0, 1
    xvv = np.einsum("bax,b->ax", P, d2)
    dl = lambda s: np.array([s - 0.5, -2.0 * s, s + 0.5])
    m_uv = max(np.linalg.norm(np.einsum("bax,a,b->x", P, dl(u), dl(v))) for u in (-1.0, 1.0) for v in (-1.0, 1.0))
    M = bern_max(xuu) + m_uv + bern_max(xvv)
    h = 1.0 / k
    return M * h * h / 4.0
