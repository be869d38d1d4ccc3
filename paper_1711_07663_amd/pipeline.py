"""One connectivity step of an overset system (background grid + bodies,
each body a wall surface and its near-body shell), on registered device
state, through the C ABI.

Step (Sec. 2.1 steps 1-2, Sec. 4.2, Sec. 4.3):
  1. cut the background by every body wall (union of holes), fringe layer;
  2. cut each shell by the other bodies' walls (posed into the shell frame);
     its overset-tagged outer faces give its fringe elements;
  3. Gauss receptor points of the background fringe -> donors in each shell;
  4. Gauss receptor points of each shell's fringe -> donors in the background.
"""
from __future__ import annotations

import numpy as np
import torch

from . import oc as _oc


def pose_inverse(p):
    R = np.asarray(p[:9], dtype=np.float64).reshape(3, 3)
    t = np.asarray(p[9:12], dtype=np.float64)
    return np.concatenate([R.T.ravel(), -R.T @ t])


def pose_compose(a, b):
    """x -> a(b(x))"""
    Ra = np.asarray(a[:9]).reshape(3, 3)
    Rb = np.asarray(b[:9]).reshape(3, 3)
    return np.concatenate([(Ra @ Rb).ravel(), Ra @ np.asarray(b[9:12]) + np.asarray(a[9:12])])


IDENTITY = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=np.float64)


class OversetSystem:
    """Registers a case (dict with ``bg`` grid and ``bodies`` [{surface,
    shell}]) on a context and keeps all per-step buffers on the device."""

    def __init__(self, ctx: _oc.Context, case, shell_points_cap=None, bg_points_cap=None):
        self.ctx = ctx
        dev = torch.device("cuda", ctx.device)
        bg = case["bg"]
        self.bg_id = ctx.register_grid(bg.nodes, bg.conn, bg.face_tags)
        self.n_bg = bg.n_elem
        self.bodies = []
        for b in case["bodies"]:
            s, sh = b["surface"], b["shell"]
            sid = ctx.register_cut_surface(s.nodes, s.conn, _oc.OC_SURF_WALL)
            gid = ctx.register_grid(sh.nodes, sh.conn, sh.face_tags)
            self.bodies.append(dict(surf=sid, shell=gid, n_shell=sh.n_elem))
        self.ib_bg = torch.empty(self.n_bg, dtype=torch.int8, device=dev)
        cap_bg = bg_points_cap or 27 * self.n_bg
        self.pts_bg = torch.empty((cap_bg, 3), dtype=torch.float64, device=dev)
        self.src_bg = torch.empty(cap_bg, dtype=torch.int32, device=dev)
        for b in self.bodies:
            n = b["n_shell"]
            cap = shell_points_cap or 27 * n
            b["ib"] = torch.empty(n, dtype=torch.int8, device=dev)
            b["pts"] = torch.empty((cap, 3), dtype=torch.float64, device=dev)
            b["src"] = torch.empty(cap, dtype=torch.int32, device=dev)
            b["donor"] = torch.empty(cap, dtype=torch.int32, device=dev)
            b["ref"] = torch.empty((cap, 3), dtype=torch.float64, device=dev)
            b["donor_bg"] = torch.empty(cap_bg, dtype=torch.int32, device=dev)
            b["ref_bg"] = torch.empty((cap_bg, 3), dtype=torch.float64, device=dev)

    def step(self, poses, stats=False):
        """Full connectivity step at the given body poses; returns counts.
        With ``stats`` the cut and donor counters of each call are collected
        too (each read synchronises the stream)."""
        ctx = self.ctx
        poses = [np.asarray(p, dtype=np.float64) for p in poses]
        sids = [b["surf"] for b in self.bodies]
        ctx.cut_multi(self.bg_id, sids, np.concatenate(poses), self.ib_bg)
        st = dict(bg_cut=ctx.last_cut_info(), donor_bg=[], donor_shell=[]) if stats else None
        for i, b in enumerate(self.bodies):
            others = [j for j in range(len(self.bodies)) if j != i]
            inv = pose_inverse(poses[i])
            rel = [pose_compose(inv, poses[j]) for j in others]
            ctx.cut_multi(b["shell"], [sids[j] for j in others], np.concatenate(rel) if rel else np.zeros(12), b["ib"])
        n_bg = ctx.fringe_points(self.bg_id, IDENTITY, self.ib_bg, self.pts_bg, self.src_bg)
        counts = dict(n_bg_points=n_bg, n_shell_points=[])
        for i, b in enumerate(self.bodies):
            ctx.donor_search(b["shell"], poses[i], self.pts_bg, n_bg, b["donor_bg"], b["ref_bg"])
            if stats:
                st["donor_bg"].append(ctx.last_donor_info())
        for i, b in enumerate(self.bodies):
            n_s = ctx.fringe_points(b["shell"], poses[i], b["ib"], b["pts"], b["src"])
            ctx.donor_search(self.bg_id, IDENTITY, b["pts"], n_s, b["donor"], b["ref"])
            counts["n_shell_points"].append(n_s)
            if stats:
                st["donor_shell"].append(ctx.last_donor_info())
        if stats:
            counts["stats"] = st
        return counts


class SlotStep:
    """The same connectivity step on a slot of an OversetSystem: poses and
    point counts live on the device, nothing synchronises, and the launch
    sequence can be captured once in a graph and replayed with new poses.

    Device pose table rows: [0, nb) body poses (background cut; shell receptor
    points and bg->shell searches); then for body i the poses of the other
    bodies in body i's frame (shell cuts); the last row is the identity."""

    def __init__(self, system: OversetSystem, stream=None):
        self.sys = system
        ctx = system.ctx
        dev = torch.device("cuda", ctx.device)
        nb = len(system.bodies)
        grids = [system.bg_id] + [b["shell"] for b in system.bodies]
        surfs = sorted(set(b["surf"] for b in system.bodies))
        cap = max([system.pts_bg.shape[0]] + [b["pts"].shape[0] for b in system.bodies])
        self.slot = ctx.create_slot(grids, surfs, cap, stream)
        self.n_pose = nb + nb * (nb - 1) + 1
        self.poses_dev = torch.zeros((self.n_pose, 12), dtype=torch.float64, device=dev)
        self.n_dev = torch.zeros(1 + nb, dtype=torch.int32, device=dev)
        self.graph = None

    def _pose_table(self, poses):
        nb = len(self.sys.bodies)
        rows = [np.asarray(p, dtype=np.float64) for p in poses]
        for i in range(nb):
            inv = pose_inverse(poses[i])
            rows += [pose_compose(inv, poses[j]) for j in range(nb) if j != i]
        rows.append(IDENTITY)
        return torch.from_numpy(np.stack(rows))

    def _launch(self):
        s, sl = self.sys, self.slot
        nb = len(s.bodies)
        sids = [b["surf"] for b in s.bodies]
        sl.cut(s.bg_id, sids, self.poses_dev[:nb], s.ib_bg)
        r = nb
        for i, b in enumerate(s.bodies):
            others = [sids[j] for j in range(nb) if j != i]
            sl.cut(b["shell"], others, self.poses_dev[r:r + nb - 1], b["ib"])
            r += nb - 1
        ident = self.poses_dev[self.n_pose - 1]
        cap_bg = s.pts_bg.shape[0]
        sl.fringe_points(s.bg_id, ident, s.ib_bg, s.pts_bg, self.n_dev[0:1], s.src_bg)
        for i, b in enumerate(s.bodies):
            sl.donor_search(b["shell"], self.poses_dev[i], s.pts_bg, cap_bg, self.n_dev[0:1], b["donor_bg"],
                            b["ref_bg"])
        for i, b in enumerate(s.bodies):
            cap = b["pts"].shape[0]
            sl.fringe_points(b["shell"], self.poses_dev[i], b["ib"], b["pts"], self.n_dev[1 + i:2 + i], b["src"])
            sl.donor_search(s.bg_id, ident, b["pts"], cap, self.n_dev[1 + i:2 + i], b["donor"], b["ref"])

    def set_poses(self, poses):
        with torch.cuda.stream(self.slot.stream):
            self.poses_dev.copy_(self._pose_table(poses))

    def step(self, poses):
        """Eager launches on the slot stream (no synchronisation)."""
        self.set_poses(poses)
        self._launch()

    def capture(self):
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.slot.set_stream(torch.cuda.current_stream())
            self._launch()
        self.slot.set_stream(self.slot.stream)
        self.graph = g
        return g

    def replay(self, poses):
        """Graph replay on the slot stream with new poses."""
        if self.graph is None:
            self.capture()
        with torch.cuda.stream(self.slot.stream):
            self.poses_dev.copy_(self._pose_table(poses))
            self.graph.replay()

    def counts(self):
        """Point counts (synchronises)."""
        n = self.n_dev.cpu().tolist()
        return dict(n_bg_points=n[0], n_shell_points=n[1:])
