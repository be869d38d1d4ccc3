"""Inputs of the connectivity-robustness cases (Sec. 4.4 and the status rule
of Sec. 4.1, Fig. multinorm), shared by the oracle pins and the GPU parity
tests.

* slot     a plate with a straight-sided slot through it, turned 45 degrees
           about z so that background nodes lie on the slot's mid-plane
           (equidistant from both slot walls, whose normals must not be
           averaged) and on the bisectors of the slot's edges;
* slot3d   the same plate at a random rotation on an anisotropic background
           (20 x 9 x 14 elements) that is itself rotated;
* groove   a block with a long narrow groove (faces of aspect ratio up to
           18) at a random pose on a background of different density per
           axis;
* wedge    a blade whose two long faces meet at a dihedral angle of 1.4e-5
           rad: the first node of element 942 lies 4e-6 from its edge, in
           the direction c b + sqrt(1 - c^2) n0 (c = 3e-5) from the nearest
           edge point, so the two nearest triangles see that node with unit
           dot products of opposite sign whose magnitudes differ by
           2 t c / sqrt(1 + t^2) = 4.2e-10 (t = 7e-6), below the 1e-9 tie
           tolerance: the side is decided by the averaged normal.
"""
import numpy as np

from workloads import meshes as M

WEDGE_T, WEDGE_C, WEDGE_DELTA = 7e-6, 3e-5, 4e-6
WEDGE_ELEMENT = 942          # first node at the origin of the 12^3 grid on [-1.5, 1.5]^3


def rotate_grid(grid, pose):
    """A copy of grid with every node moved by the rigid pose."""
    return M.Grid(nodes=M.apply_pose_to_points(pose, grid.nodes), conn=grid.conn.copy(),
                  face_tags=None if grid.face_tags is None else grid.face_tags.copy(),
                  name=grid.name + " (rotated)", shape=grid.shape)


def case(name):
    """(background grid, surface, surface pose)"""
    if name == "slot":
        return (M.background_grid(12, -1.5, 1.5, amp=0.0), M.slotted_plate(w=0.4, c=0.35),
                M.pose_rz(np.pi / 4))
    if name == "slot3d":
        rng = np.random.default_rng(4401)
        bg = rotate_grid(M.background_grid((20, 9, 14), -1.6, 1.6, amp=0.0), M.random_pose(rng, 0.05))
        return bg, M.slotted_plate(w=0.3, c=0.3, k=3), M.random_pose(rng, 0.1)
    if name == "groove":
        rng = np.random.default_rng(4402)
        bg = M.background_grid((11, 23, 16), -1.6, 1.6, amp=0.01)
        return bg, M.grooved_block(a=1.1, b=0.9, c=0.45, w=0.05, depth=0.3, k=1), M.random_pose(rng, 0.1)
    if name == "wedge":
        e = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
        n0 = np.ones(3) / np.sqrt(3.0)
        b = np.cross(n0, e)
        sn = np.sqrt(1.0 - WEDGE_C * WEDGE_C)
        apex = -WEDGE_DELTA * (WEDGE_C * b + sn * n0)
        return (M.background_grid(12, -1.5, 1.5, amp=0.0), M.thin_wedge(apex, e, b, WEDGE_T, 0.2, 0.6),
                M.IDENTITY_POSE.copy())
    raise KeyError(name)


NAMES = ("slot", "slot3d", "groove", "wedge")
