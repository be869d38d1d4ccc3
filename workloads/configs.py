"""The five benchmark workloads and smaller test cases, built from seeds.

Every case is a dict with a background grid ``bg``, a list of ``bodies`` (each a
cut surface of kind wall plus its near-body shell) and the per-body poses.

* tiny        16^3 background on [-2,2]^3, R = 0.5 cube-sphere of 96 faces,
              4-layer shell to r = 1.
* dimpled     128^3 background on [-3,3]^3, 300-dimple sphere of 24 576 faces,
              8-layer shell to r = 1.
* spinning    the dimpled case rotating about z at one turn per 400 steps.
* moving      the dimpled case turning about z and oscillating along x
              (amplitude 0.5), for the unblanking of a moving body.
* batch64     64 uneven instances drawn from SeedSequence(1711).
* two-body    two dimpled spheres 1.5 apart on a 160^3 background.
"""
from __future__ import annotations

import math

import numpy as np

from . import meshes as M

DIMPLE_A = 0.04
DIMPLE_K = 0.008


def make_case(bg_n, bg_lo, bg_hi, m, layers, R=0.5, dimples=0, axes=None, amp=0.02,
              r_out=1.0, scale_out=None, name="case"):
    bg = M.background_grid(bg_n, bg_lo, bg_hi, amp=amp, name=name + "/bg")
    surf = M.cube_sphere(m, R=R, axes=axes, dimples=dimples, dimple_a=DIMPLE_A,
                         dimple_k=DIMPLE_K, name=name + "/wall")
    shell = M.shell_grid(surf, layers, r_out=r_out, scale_out=scale_out, name=name + "/shell")
    return dict(name=name, bg=bg, bodies=[dict(surface=surf, shell=shell,
                                               boundary=M.shell_boundary(shell, surf, name + "/boundary"))],
                poses=[M.IDENTITY_POSE.copy()])


def tiny():
    """16^3 quadratic hexes on [-2,2]^3 with the sinusoidal displacement, a
    96-face R = 0.5 cube-sphere and its 4-layer shell."""
    return make_case(16, -2.0, 2.0, m=4, layers=4, name="tiny")


def dimpled(bg_n=128, m=64, layers=8, dimples=300):
    """Single cut of the 300-dimple sphere on a 128^3 background on [-3,3]^3."""
    return make_case(bg_n, -3.0, 3.0, m=m, layers=layers, dimples=dimples, name="dimpled")


def spinning_poses(n_steps=200, steps_per_rev=400):
    """Poses R_z(2 pi n / steps_per_rev), n = 1..n_steps."""
    return [M.pose_rz(2.0 * math.pi * n / steps_per_rev) for n in range(1, n_steps + 1)]


def moving_poses(n_steps=200, steps_per_rev=400, amp=0.5):
    """Poses of a body turning about z at one turn per steps_per_rev steps
    while oscillating along x with amplitude amp: R_z(2 pi n / steps_per_rev),
    t = (amp sin(2 pi n / steps_per_rev), 0, 0), n = 0..n_steps."""
    out = []
    for n in range(n_steps + 1):
        th = 2.0 * math.pi * n / steps_per_rev
        out.append(M.pose_rz(th, (amp * math.sin(th), 0.0, 0.0)))
    return out


def batch_instances(n=64, seed=1711, n_lo=16, n_hi=96, m_lo=8, m_hi=64):
    """Uneven instances: background n log-uniform in [n_lo, n_hi] on [-2,2]^3,
    body in {sphere, ellipsoid 0.5/0.35/0.25, dimpled sphere with 50..300
    dimples}, faces per cube edge log-uniform in [m_lo, m_hi], random SO(3)
    rotation and a translation within +-0.3."""
    seqs = np.random.SeedSequence(seed).spawn(n)
    out = []
    for i, s in enumerate(seqs):
        rng = np.random.default_rng(s)
        bn = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        kind = int(rng.integers(0, 3))
        nd = int(rng.integers(50, 301))
        pose = M.random_pose(rng, 0.3)
        out.append(dict(index=i, bg_n=bn, m=m, kind=("sphere", "ellipsoid", "dimpled")[kind],
                        dimples=nd if kind == 2 else 0, pose=pose))
    return out


def batch_case(spec, layers=4):
    axes = (0.5, 0.35, 0.25) if spec["kind"] == "ellipsoid" else None
    c = make_case(spec["bg_n"], -2.0, 2.0, m=spec["m"], layers=layers,
                  dimples=spec["dimples"], axes=axes, scale_out=2.0,
                  name="batch%02d" % spec["index"])
    c["poses"] = [np.asarray(spec["pose"], dtype=np.float64)]
    return c


def two_body(bg_n=160, m=64, layers=8, dimples=300):
    """Two dimpled spheres centred at (+-0.75, 0, 0) on a bg_n^3 background on
    [-3,3]^3; each body's shell reaches r = 1 and so touches the other sphere."""
    bg = M.background_grid(bg_n, -3.0, 3.0, amp=0.02, name="two-body/bg")
    surf = M.cube_sphere(m, R=0.5, dimples=dimples, dimple_a=DIMPLE_A, dimple_k=DIMPLE_K,
                         name="two-body/wall")
    shell = M.shell_grid(surf, layers, r_out=1.0, name="two-body/shell")
    bnd = M.shell_boundary(shell, surf, "two-body/boundary")
    bodies = [dict(surface=surf, shell=shell, boundary=bnd), dict(surface=surf, shell=shell, boundary=bnd)]
    poses = [M.pose_rz(0.0, (-0.75, 0.0, 0.0)), M.pose_rz(0.0, (0.75, 0.0, 0.0))]
    return dict(name="two-body", bg=bg, bodies=bodies, poses=poses)


def two_body_poses(step, steps_per_rev=400):
    th = 2.0 * math.pi * step / steps_per_rev
    return [M.pose_rz(th, (-0.75, 0.0, 0.0)), M.pose_rz(-th, (0.75, 0.0, 0.0))]
