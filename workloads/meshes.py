"""Seeded synthetic geometry for the overset connectivity workloads.

This module only builds inputs: node coordinates, connectivity, face tags and
poses.  It holds none of the method's arithmetic (no shape functions, no
distances, no classification), so both the CPU oracle and the HIP path can take
their inputs from here without sharing any step of the method.

Conventions (the paper's isoparametric hexahedra, Sec. 4.3, eq. reftophys):

* A quadratic hexahedron has 27 nodes on the reference lattice {-1, 0, 1}^3,
  local index ``a + 3*b + 9*c`` for (xi, eta, zeta) indices (a, b, c).
* A quadratic surface face has 9 nodes, local index ``a + 3*b``; the outward
  normal is d/dxi x d/deta (right-handed).
* Face tags per element, order (-xi, +xi, -eta, +eta, -zeta, +zeta):
  0 interior, 1 wall, 2 overset, 3 far field.
* A pose is 12 doubles: the row-major rotation R followed by the offset t,
  applied as x' = R x + t.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

TAG_INTERIOR, TAG_WALL, TAG_OVERSET, TAG_FARFIELD = 0, 1, 2, 3


@dataclass
class Grid:
    """Quadratic hexahedral grid: unique nodes + 27-node connectivity."""
    nodes: np.ndarray            # (n_nodes, 3) float64
    conn: np.ndarray             # (n_elem, 27) int32
    face_tags: np.ndarray | None = None   # (n_elem, 6) int8
    name: str = ""
    shape: tuple = ()            # (nx, ny, nz) for structured background grids

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])


@dataclass
class Surface:
    """Closed surface of 9-node quadratic quads (outward oriented)."""
    nodes: np.ndarray            # (n_nodes, 3) float64
    conn: np.ndarray             # (n_face, 9) int32
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_face(self) -> int:
        return int(self.conn.shape[0])


# --------------------------------------------------------------------------
# background grids
# --------------------------------------------------------------------------

def background_grid(n, lo=-2.0, hi=2.0, amp=0.02, name="background"):
    """n^3 (or nx*ny*nz) quadratic hexes on the box [lo, hi]^3.

    The node lattice has 2n+1 equispaced planes per axis.  Every node is moved
    by the same scalar ``amp*sin(pi x) sin(pi y) sin(pi z)`` added to each of its
    three coordinates, which curves the element faces.
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    ax = [lo + np.arange(2 * m + 1, dtype=np.float64) * ((hi - lo) / (2 * m))
          for m in (nx, ny, nz)]
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    # node index I + NX*J + NX*NY*K  -> array order (K, J, I)
    X = X.transpose(2, 1, 0).ravel()
    Y = Y.transpose(2, 1, 0).ravel()
    Z = Z.transpose(2, 1, 0).ravel()
    if amp != 0.0:
        s = amp * np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        X = X + s
        Y = Y + s
        Z = Z + s
    nodes = np.stack([X, Y, Z], axis=1)
    NX, NY = 2 * nx + 1, 2 * ny + 1
    i = np.arange(nx)
    j = np.arange(ny)
    k = np.arange(nz)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")       # element id i + nx*j + nx*ny*k
    I = I.ravel(); J = J.ravel(); K = K.ravel()
    conn = np.empty((I.size, 27), dtype=np.int64)
    for c in range(3):
        for b in range(3):
            for a in range(3):
                conn[:, a + 3 * b + 9 * c] = (2 * I + a) + NX * (2 * J + b) + NX * NY * (2 * K + c)
    return Grid(nodes=nodes, conn=conn.astype(np.int32), face_tags=None, name=name,
                shape=(nx, ny, nz))


# --------------------------------------------------------------------------
# cube-sphere surfaces
# --------------------------------------------------------------------------

def _cube_lattice(m):
    """Unique integer points of the boundary of the cube [0, 2m]^3 and the
    9-node face connectivity of the 6*m*m quadratic faces (outward)."""
    N = 2 * m
    keys = {}
    pts = []

    def idx(I, J, K):
        key = (I, J, K)
        v = keys.get(key)
        if v is None:
            v = len(pts)
            keys[key] = v
            pts.append(key)
        return v

    # (U, V) -> (I, J, K) per cube face with d/dU x d/dV pointing outward
    maps = [
        lambda U, V: (N, U, V),      # +x : y x z = +x
        lambda U, V: (0, V, U),      # -x : z x y = -x
        lambda U, V: (V, N, U),      # +y : z x x = +y
        lambda U, V: (U, 0, V),      # -y : x x z = -y
        lambda U, V: (U, V, N),      # +z : x x y = +z
        lambda U, V: (V, U, 0),      # -z : y x x = -z
    ]
    conn = []
    for f in maps:
        for fj in range(m):
            for fi in range(m):
                face = []
                for q in range(3):
                    for p in range(3):
                        face.append(idx(*f(2 * fi + p, 2 * fj + q)))
                conn.append(face)
    lat = np.array(pts, dtype=np.float64)
    return lat, np.array(conn, dtype=np.int32)


def fibonacci_centres(n):
    """Fibonacci lattice of n unit vectors: z_i = 1 - (2i+1)/n, phi_i = i*pi*(3-sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _dimple_radius(dirs, R, centres, a, k):
    """Radius along unit rays ``dirs`` of a sphere of radius R carrying
    spherical-cap dimples of chord radius a and depth k at ``centres``."""
    rho = (a * a + k * k) / (2.0 * k)
    C = (R - k + rho) * centres                    # cap-sphere centres
    r = np.full(dirs.shape[0], R)
    cc = np.einsum("ij,ij->i", C, C)
    for s in range(0, dirs.shape[0], 4096):
        d = dirs[s:s + 4096]
        b = d @ C.T                                   # (n, nd)
        disc = b * b - cc[None, :] + rho * rho
        ok = (disc >= 0.0) & (b > 0.0)
        t = np.where(ok, b - np.sqrt(np.where(ok, disc, 0.0)), np.inf)
        t = np.where(t < R, t, np.inf)
        tmin = t.min(axis=1)
        r[s:s + 4096] = np.where(np.isfinite(tmin), tmin, R)
    return r


def cube_sphere(m, R=0.5, axes=None, dimples=0, dimple_a=0.04, dimple_k=0.008,
                name="sphere"):
    """Closed cube-sphere of 6*m*m 9-node quads.

    Gnomonic construction: cube-face points on an equispaced (2m+1)^2 lattice
    are normalised onto the unit sphere.  ``axes`` scales to an ellipsoid;
    ``dimples`` > 0 carves spherical-cap dimples centred on a Fibonacci lattice.
    """
    lat, conn = _cube_lattice(m)
    c = lat / m - 1.0                                  # cube coordinates in [-1, 1]
    dirs = c / np.sqrt((c * c).sum(axis=1))[:, None]
    if dimples:
        cen = fibonacci_centres(dimples)
        r = _dimple_radius(dirs, R, cen, dimple_a, dimple_k)
    else:
        r = np.full(dirs.shape[0], R)
    nodes = dirs * r[:, None]
    if axes is not None:
        nodes = dirs * np.asarray(axes, dtype=np.float64)[None, :]
    meta = dict(m=m, R=R, axes=axes, dimples=dimples)
    return Surface(nodes=nodes, conn=conn, name=name, meta=meta)


def box_surface(m, lo, hi, name="box"):
    """Axis-aligned box [lo, hi]^3 made of flat 9-node quads (m per edge)."""
    lat, conn = _cube_lattice(m)
    lo = np.asarray(lo, dtype=np.float64) * np.ones(3)
    hi = np.asarray(hi, dtype=np.float64) * np.ones(3)
    nodes = lo[None, :] + (hi - lo)[None, :] * (lat / (2.0 * m))
    return Surface(nodes=nodes, conn=conn, name=name, meta=dict(m=m, lo=lo, hi=hi))


# --------------------------------------------------------------------------
# flat-faced solids from patches (slots, grooves, thin wedges)
# --------------------------------------------------------------------------

def patch_surface(corners, patches, k=1, name="patches"):
    """Closed surface of 9-node quads from flat quadrilateral patches.

    ``corners`` (nc, 3) and ``patches`` [(i00, i10, i11, i01)] of corner ids,
    each ordered so that (c10 - c00) x (c01 - c00) points out of the solid.
    Every patch becomes k x k quadratic faces on a (2k+1)^2 node lattice.
    Points on a patch edge are interpolated from the edge's two corners in
    ascending id order, so two patches sharing an edge share its nodes bit
    for bit (the surface is watertight when every patch edge is shared)."""
    corners = np.asarray(corners, dtype=np.float64)
    N = 2 * k
    keys = {}
    pts = []

    def node(key, xyz):
        v = keys.get(key)
        if v is None:
            v = len(pts)
            keys[key] = v
            pts.append(xyz)
        return v

    def edge_point(a, b, m):
        # point m of N along the edge from corner a to corner b
        if m == 0:
            return node(("c", a), corners[a])
        if m == N:
            return node(("c", b), corners[b])
        lo, hi, mm = (a, b, m) if a < b else (b, a, N - m)
        t = mm / N
        return node(("e", lo, hi, mm), (1.0 - t) * corners[lo] + t * corners[hi])

    conn = []
    for pi_, (c00, c10, c11, c01) in enumerate(patches):
        P00, P10, P11, P01 = corners[c00], corners[c10], corners[c11], corners[c01]
        lat = np.empty((N + 1, N + 1), dtype=np.int64)
        for j in range(N + 1):
            for i in range(N + 1):
                if j == 0:
                    lat[i, j] = edge_point(c00, c10, i)
                elif j == N:
                    lat[i, j] = edge_point(c01, c11, i)
                elif i == 0:
                    lat[i, j] = edge_point(c00, c01, j)
                elif i == N:
                    lat[i, j] = edge_point(c10, c11, j)
                else:
                    u, v = i / N, j / N
                    xyz = ((1 - u) * (1 - v)) * P00 + (u * (1 - v)) * P10 + (u * v) * P11 + ((1 - u) * v) * P01
                    lat[i, j] = node(("i", pi_, i, j), xyz)
        for fj in range(k):
            for fi in range(k):
                conn.append([lat[2 * fi + a, 2 * fj + b] for b in range(3) for a in range(3)])
    return Surface(nodes=np.array(pts, dtype=np.float64), conn=np.array(conn, dtype=np.int32), name=name,
                   meta=dict(k=k))


def voxel_solid_surface(xs, ys, zs, solid, k=1, name="voxels"):
    """Boundary of a union of cells of the rectilinear lattice xs x ys x zs
    (solid[i, j, l] True = cell filled) as a closed surface of flat 9-node
    quads, k x k per cell face, oriented outward."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    solid = np.asarray(solid, dtype=bool)
    nx, ny, nz = solid.shape
    cid = lambda i, j, l: i + (nx + 1) * (j + (ny + 1) * l)
    corners = np.array([(xs[i], ys[j], zs[l]) for l in range(nz + 1) for j in range(ny + 1)
                        for i in range(nx + 1)], dtype=np.float64)

    def filled(i, j, l):
        return 0 <= i < nx and 0 <= j < ny and 0 <= l < nz and solid[i, j, l]

    patches = []
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                if not solid[i, j, l]:
                    continue
                if not filled(i + 1, j, l):   # +x: edges along y then z
                    patches.append((cid(i + 1, j, l), cid(i + 1, j + 1, l), cid(i + 1, j + 1, l + 1), cid(i + 1, j, l + 1)))
                if not filled(i - 1, j, l):   # -x
                    patches.append((cid(i, j, l), cid(i, j, l + 1), cid(i, j + 1, l + 1), cid(i, j + 1, l)))
                if not filled(i, j + 1, l):   # +y: edges along z then x
                    patches.append((cid(i, j + 1, l), cid(i, j + 1, l + 1), cid(i + 1, j + 1, l + 1), cid(i + 1, j + 1, l)))
                if not filled(i, j - 1, l):   # -y
                    patches.append((cid(i, j, l), cid(i + 1, j, l), cid(i + 1, j, l + 1), cid(i, j, l + 1)))
                if not filled(i, j, l + 1):   # +z: edges along x then y
                    patches.append((cid(i, j, l + 1), cid(i + 1, j, l + 1), cid(i + 1, j + 1, l + 1), cid(i, j + 1, l + 1)))
                if not filled(i, j, l - 1):   # -z
                    patches.append((cid(i, j, l), cid(i, j + 1, l), cid(i + 1, j + 1, l), cid(i + 1, j, l)))
    surf = patch_surface(corners, patches, k, name)
    surf.meta.update(xs=xs, ys=ys, zs=zs)
    return surf


def slotted_plate(a=1.0, b=0.8, c=0.35, w=0.3, s=0.5, k=2, name="slotted plate"):
    """A plate [-a,a] x [-b,b] x [-c,c] with a straight-sided slot |x| < w,
    |y| < s cut through it along z (the slot test of Sec. 4.4): a closed
    genus-one surface of flat faces."""
    solid = np.ones((3, 3, 1), dtype=bool)
    solid[1, 1, 0] = False
    return voxel_solid_surface([-a, -w, w, a], [-b, -s, s, b], [-c, c], solid, k, name)


def grooved_block(a=1.0, b=0.8, c=0.5, w=0.2, depth=0.35, k=2, name="grooved block"):
    """A block [-a,a] x [-b,b] x [-c,c] with a groove |x| < w, z > c - depth
    cut along its whole length in y (a concave channel, Sec. 4.4)."""
    solid = np.ones((3, 1, 2), dtype=bool)
    solid[1, 0, 1] = False
    return voxel_solid_surface([-a, -w, w, a], [-b, b], [-c, c - depth, c], solid, k, name)


def thin_wedge(apex, e, b, t, L, U, k=1, name="thin wedge"):
    """A thin triangular prism (a blade): cross-section triangle with apex
    at ``apex``, opening towards -b with half-thickness t per unit length
    (vertices apex, apex - L b +- t L n0, n0 = e x b), extruded along the unit
    vector e over [-U, U].  The two long faces meet at the apex edge at a
    dihedral angle of about 2t; their outward normals are nearly opposite."""
    e = np.asarray(e, dtype=np.float64) / np.linalg.norm(e)
    b = np.asarray(b, dtype=np.float64)
    b = b - e * (b @ e)
    b /= np.linalg.norm(b)
    n0 = np.cross(e, b)
    apex = np.asarray(apex, dtype=np.float64)
    sec = dict(A=(0.0, 0.0), B=(-L, t * L), C=(-L, -t * L))     # (b, n0) coordinates, counter-clockwise
    sec["Mab"] = tuple(0.5 * (np.array(sec["A"]) + np.array(sec["B"])))
    sec["Mbc"] = tuple(0.5 * (np.array(sec["B"]) + np.array(sec["C"])))
    sec["Mca"] = tuple(0.5 * (np.array(sec["C"]) + np.array(sec["A"])))
    sec["G"] = tuple((np.array(sec["A"]) + np.array(sec["B"]) + np.array(sec["C"])) / 3.0)
    names = ["A", "Mab", "B", "Mbc", "C", "Mca", "G"]
    corners, cid = [], {}
    for side, g in (("-", -U), ("+", U)):
        for nm in names:
            cid[nm + side] = len(corners)
            corners.append(apex + sec[nm][0] * b + sec[nm][1] * n0 + g * e)
    ring = ["A", "Mab", "B", "Mbc", "C", "Mca"]
    patches = []
    for i in range(6):
        p, q = ring[i], ring[(i + 1) % 6]
        patches.append((cid[p + "-"], cid[q + "-"], cid[q + "+"], cid[p + "+"]))
    for quad in (("A", "Mab", "G", "Mca"), ("B", "Mbc", "G", "Mab"), ("C", "Mca", "G", "Mbc")):
        patches.append(tuple(cid[nm + "+"] for nm in quad))
        patches.append(tuple(cid[nm + "-"] for nm in (quad[0], quad[3], quad[2], quad[1])))
    surf = patch_surface(np.array(corners), patches, k, name)
    surf.meta.update(apex=apex, e=e, b=b, n0=n0, t=t, L=L, U=U)
    return surf


# --------------------------------------------------------------------------
# near-body shells
# --------------------------------------------------------------------------

def shell_grid(surf: Surface, layers, r_out=1.0, scale_out=None, name="shell"):
    """Near-body grid of quadratic hexes extruded radially from a surface.

    Each surface node moves along its ray from the origin; levels 0..2L are
    equally spaced from the surface to radius ``r_out`` (or to ``scale_out``
    times the surface radius).  The inner (-zeta) faces are tagged wall and
    the outer (+zeta) faces overset.  Element id = layer * n_face + face.
    """
    ps = surf.nodes
    rs = np.sqrt((ps * ps).sum(axis=1))
    nlev = 2 * layers + 1
    ns = ps.shape[0]
    nodes = np.empty((nlev * ns, 3), dtype=np.float64)
    for l in range(nlev):
        f = l / (2.0 * layers)
        if scale_out is None:
            fac = 1.0 + (r_out / rs - 1.0) * f
        else:
            fac = 1.0 + (scale_out - 1.0) * f
        nodes[l * ns:(l + 1) * ns] = ps * fac[:, None] if np.ndim(fac) else ps * fac
    nf = surf.n_face
    conn = np.empty((layers * nf, 27), dtype=np.int64)
    tags = np.zeros((layers * nf, 6), dtype=np.int8)
    for lay in range(layers):
        e0 = lay * nf
        for c in range(3):
            lev = 2 * lay + c
            for q in range(9):
                conn[e0:e0 + nf, q + 9 * c] = lev * ns + surf.conn[:, q]
    tags[:nf, 4] = TAG_WALL
    tags[(layers - 1) * nf:, 5] = TAG_OVERSET
    return Grid(nodes=nodes, conn=conn.astype(np.int32), face_tags=tags, name=name)


def shell_boundary(shell: Grid, surf: Surface, name="boundary"):
    """The outer (overset) boundary of a near-body grid made by shell_grid,
    as a closed cut surface: the outermost node level (the same coordinates
    as the grid's outer faces) with the wall's face connectivity, so it is
    oriented outward like the wall."""
    ns = surf.nodes.shape[0]
    nlev = shell.nodes.shape[0] // ns
    return Surface(nodes=np.ascontiguousarray(shell.nodes[(nlev - 1) * ns:]), conn=surf.conn.copy(), name=name)


# --------------------------------------------------------------------------
# poses
# --------------------------------------------------------------------------

IDENTITY_POSE = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=np.float64)


def pose_rz(theta, t=(0.0, 0.0, 0.0)):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([c, -s, 0.0, s, c, 0.0, 0.0, 0.0, 1.0, t[0], t[1], t[2]], dtype=np.float64)


def pose_from_quaternion(q, t=(0.0, 0.0, 0.0)):
    w, x, y, z = (float(v) for v in np.asarray(q, dtype=np.float64) / np.linalg.norm(q))
    R = [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]
    return np.array(R + list(t), dtype=np.float64)


def random_pose(rng, trans=0.3):
    """Uniform rotation on SO(3) (uniform unit quaternion) and a translation
    drawn from U(-trans, trans)^3."""
    q = rng.standard_normal(4)
    t = rng.uniform(-trans, trans, 3)
    return pose_from_quaternion(q, t)


def apply_pose_to_points(pose, pts):
    """x' = R x + t (used to build posed copies of inputs, e.g. rigid-motion tests)."""
    R = np.asarray(pose[:9], dtype=np.float64).reshape(3, 3)
    return pts @ R.T + np.asarray(pose[9:12], dtype=np.float64)[None, :]


def compose_pose(a, b):
    """Pose of x -> a(b(x))."""
    Ra = np.asarray(a[:9]).reshape(3, 3)
    Rb = np.asarray(b[:9]).reshape(3, 3)
    R = Ra @ Rb
    t = Ra @ np.asarray(b[9:12]) + np.asarray(a[9:12])
    return np.concatenate([R.ravel(), t])
