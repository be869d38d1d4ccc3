"""One connectivity step of an overset system (background grid + bodies,
each body a wall surface and its near-body shell), on registered device
state, through the C ABI.

Step (Sec. 2.1 steps 1-2, Sec. 4.2, Sec. 4.3):
  1. cut the background by every body wall (union of holes), fringe layer;
  2. cut each shell by the other bodies' walls (posed into the shell frame);
     its overset-tagged outer faces give its fringe elements;
  3. Gauss receptor points of the background fringe -> donors in each shell;
  4. Gauss receptor points of each shell's fringe -> donors in the background.

SlotStep(ab=True) takes the receptors of the artificial-boundary method
(Sec. 2) instead: the flux points of each grid's AB faces (faces between a
kept cell and a hole, and a shell's overset outer faces), their donors, and
the interpolation weights of the donor's solution basis at each receptor.
"""
from __future__ import annotations

import numpy as np
import torch

from . import oc as _oc


IDENTITY = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=np.float64)


class OversetSystem:
    """Registers a case (dict with ``bg`` grid and ``bodies`` [{surface,
    shell}]) on a context and keeps all per-step buffers on the device."""

    def __init__(self, ctx: _oc.Context, case, shell_points_cap=None, bg_points_cap=None, topology="walls"):
        """topology "walls": the background is cut by the bodies' walls;
        "paper": by each near-body grid's overset outer boundary (Sec. 3:
        background elements enclosed by another grid's overset boundary are
        removed), the shells by the other bodies' walls."""
        if topology not in ("walls", "paper"):
            raise ValueError("topology must be 'walls' or 'paper'")
        self.ctx = ctx
        self.topology = topology
        dev = torch.device("cuda", ctx.device)
        bg = case["bg"]
        self.bg_id = ctx.register_grid(bg.nodes, bg.conn, bg.face_tags)
        self.n_bg = bg.n_elem
        self.bodies = []
        for b in case["bodies"]:
            s, sh = b["surface"], b["shell"]
            sid = ctx.register_cut_surface(s.nodes, s.conn, _oc.OC_SURF_WALL)
            gid = ctx.register_grid(sh.nodes, sh.conn, sh.face_tags)
            n_tagged = 0 if sh.face_tags is None else int((np.asarray(sh.face_tags) == _oc.OC_FACE_OVERSET).sum())
            d = dict(surf=sid, shell=gid, n_shell=sh.n_elem, n_tagged=n_tagged)
            if topology == "paper":
                bnd = b["boundary"]
                d["bsurf"] = ctx.register_cut_surface(bnd.nodes, bnd.conn, _oc.OC_SURF_OVERSET)
            self.bodies.append(d)
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

    def bg_cutters(self):
        """Surface ids that cut the background, one per body."""
        return [b["bsurf"] if self.topology == "paper" else b["surf"] for b in self.bodies]

    def step(self, poses, stats=False):
        """Full connectivity step at the given body poses; returns counts.
        With ``stats`` the cut and donor counters of each call are collected
        too (each read synchronises the stream)."""
        ctx = self.ctx
        poses = [np.asarray(p, dtype=np.float64) for p in poses]
        sids = [b["surf"] for b in self.bodies]
        ctx.cut_multi(self.bg_id, self.bg_cutters(), np.concatenate(poses), self.ib_bg)
        st = dict(bg_cut=ctx.last_cut_info(), donor_bg=[], donor_shell=[]) if stats else None
        for i, b in enumerate(self.bodies):
            # the shell moves with its body: the library composes the other
            # walls' world poses into the shell's frame
            others = [j for j in range(len(self.bodies)) if j != i]
            ctx.cut_posed(b["shell"], poses[i], [sids[j] for j in others],
                          np.concatenate([poses[j] for j in others]) if others else np.zeros(12), b["ib"])
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


def _alloc_outputs(system, dev, n_ib_bg=1):
    """Device output buffers of one connectivity step of ``system``."""
    out = dict(ib_bg=[torch.empty(system.n_bg, dtype=torch.int8, device=dev) for _ in range(n_ib_bg)])
    cap_bg = system.pts_bg.shape[0]
    out["pts_bg"] = torch.empty((cap_bg, 3), dtype=torch.float64, device=dev)
    out["src_bg"] = torch.empty(cap_bg, dtype=torch.int32, device=dev)
    out["bodies"] = []
    for b in system.bodies:
        cap = b["pts"].shape[0]
        out["bodies"].append(dict(
            ib=torch.empty(b["n_shell"], dtype=torch.int8, device=dev),
            pts=torch.empty((cap, 3), dtype=torch.float64, device=dev),
            src=torch.empty(cap, dtype=torch.int32, device=dev),
            donor=torch.empty(cap, dtype=torch.int32, device=dev),
            ref=torch.empty((cap, 3), dtype=torch.float64, device=dev),
            donor_bg=torch.empty(cap_bg, dtype=torch.int32, device=dev),
            ref_bg=torch.empty((cap_bg, 3), dtype=torch.float64, device=dev)))
    return out


def _alloc_ab_outputs(system, dev, n_ib_bg, faces_bg_cap, faces_sh_caps, m):
    """Device output buffers of one AB step: face ids, m*m flux points per
    face, donors and m^3 weights per point."""
    mm, m3 = m * m, m ** 3
    cap_bg = faces_bg_cap * mm
    out = dict(ib_bg=[torch.empty(system.n_bg, dtype=torch.int8, device=dev) for _ in range(n_ib_bg)],
               faces_bg=torch.empty(faces_bg_cap, dtype=torch.int32, device=dev),
               pts_bg=torch.empty((cap_bg, 3), dtype=torch.float64, device=dev),
               src_bg=torch.empty(cap_bg, dtype=torch.int32, device=dev), bodies=[])
    for b, fcap in zip(system.bodies, faces_sh_caps):
        cap = fcap * mm
        out["bodies"].append(dict(
            ib=torch.empty(b["n_shell"], dtype=torch.int8, device=dev),
            faces=torch.empty(fcap, dtype=torch.int32, device=dev),
            pts=torch.empty((cap, 3), dtype=torch.float64, device=dev),
            src=torch.empty(cap, dtype=torch.int32, device=dev),
            donor=torch.empty(cap, dtype=torch.int32, device=dev),
            ref=torch.empty((cap, 3), dtype=torch.float64, device=dev),
            w=torch.empty((cap, m3), dtype=torch.float64, device=dev),
            donor_bg=torch.empty(cap_bg, dtype=torch.int32, device=dev),
            ref_bg=torch.empty((cap_bg, 3), dtype=torch.float64, device=dev),
            w_bg=torch.empty((cap_bg, m3), dtype=torch.float64, device=dev)))
    return out


class SlotStep:
    """The connectivity step of an OversetSystem on slots of its own: poses
    and point counts live on the device, the outputs belong to this object
    (several SlotSteps of one system can run at once), nothing synchronises,
    and the launch sequence can be captured in a graph and replayed with new
    poses.

    The step is two independent chains, each on its own slot and stream:
      A  background cut by every wall -> background receptor points -> their
         donors in every shell;
      B  each shell cut by the other walls -> shell receptor points -> their
         donors in the background.
    Chain B forks from A's stream after the pose upload and joins it at the
    end, so the latency-bound cut kernels of A overlap B's donor search (also
    inside a captured graph).  Chain A, the longer one, is issued first.

    Device pose table rows (world frame): [0, nb) body poses (background
    cut; shell receptor points and bg->shell searches); then for body i the
    poses of the other bodies, in order (shell cuts: the library composes
    them into body i's frame on the device); the last row is the identity.

    ``warm``: (one body) the background cut of step k starts from the iblank
    of step k-1 with the sweep bound ``sweep`` (a bound on how far any wall
    point moves in one step, e.g. Context.sweep_bound of two consecutive
    poses); the two iblank buffers alternate, so a captured step exists for
    each parity.  A warm step whose pose lies farther than ``sweep`` from
    the previous step's (checked on the host poses given to ``step``,
    ``replay`` and ``replay_table`` with a host table) runs as an eager cold
    step instead; a device pose table is not read back, so its caller keeps
    consecutive poses within ``sweep``."""

    def __init__(self, system: OversetSystem, stream=None, warm=False, sweep=0.0, ab=False, ab_faces_cap=None,
                 nodes1d=_oc.GAUSS3):
        self.sys = system
        ctx = system.ctx
        dev = torch.device("cuda", ctx.device)
        nb = len(system.bodies)
        if warm and nb != 1:
            raise ValueError("warm start needs exactly one body")
        grids = [system.bg_id] + [b["shell"] for b in system.bodies]
        surfs = [b["surf"] for b in system.bodies] + (system.bg_cutters() if system.topology == "paper" else [])
        self.ab = ab
        self.nodes1d = tuple(float(v) for v in nodes1d)
        if ab:
            m = len(self.nodes1d)
            if ab_faces_cap is None:
                ab_faces_cap = [system.pts_bg.shape[0] // (m * m)] + [2 * b["n_tagged"] + 8192 for b in system.bodies]
            self.out = _alloc_ab_outputs(system, dev, 2 if warm else 1, ab_faces_cap[0], ab_faces_cap[1:], m)
            cap = max([self.out["pts_bg"].shape[0]] + [b["pts"].shape[0] for b in self.out["bodies"]])
        else:
            self.out = _alloc_outputs(system, dev, 2 if warm else 1)
            cap = max([system.pts_bg.shape[0]] + [b["pts"].shape[0] for b in system.bodies])
        self.slot = ctx.create_slot(grids, surfs, cap, stream)
        self.slot_b = ctx.create_slot(grids, surfs, cap)
        self.n_pose = nb + nb * (nb - 1) + 1
        self.poses_dev = torch.zeros((self.n_pose, 12), dtype=torch.float64, device=dev)
        self.n_dev = torch.zeros(1 + nb, dtype=torch.int32, device=dev)
        self.nf_dev = torch.zeros(1 + nb, dtype=torch.int32, device=dev)
        self.warm = warm
        self.sweep = float(sweep)
        self.k = 0              # steps launched (selects the iblank buffer when warm)
        self.graphs = {}
        self._last_pose = None  # host pose of the last warm-checked step (None: unknown)
        self.cold_fallbacks = 0  # warm steps run cold because the pose moved too far
        self._capture_forks = 0  # stream forks issued inside the current capture

    @property
    def stream(self):
        return self.slot.stream

    def close(self):
        self.slot.close()
        self.slot_b.close()

    def nbytes(self):
        return self.slot.nbytes() + self.slot_b.nbytes()

    def ib_bg(self, k=None):
        """Background iblank of step k (default: the last launched step)."""
        bufs = self.out["ib_bg"]
        k = self.k - 1 if k is None else k
        return bufs[k % len(bufs)]

    def _pose_table(self, poses):
        nb = len(self.sys.bodies)
        rows = [np.asarray(p, dtype=np.float64) for p in poses]
        for i in range(nb):
            rows += [rows[j] for j in range(nb) if j != i]
        rows.append(IDENTITY)
        return torch.from_numpy(np.stack(rows))

    def _launch(self, k, cold, main=None, serial=False):
        """Both chains; ``main`` is the stream chain A runs on (the slot's
        own stream, or the capture stream).  ``serial`` runs chain B on the
        main stream too (no overlap: every kernel has the device to itself,
        for per-kernel timing)."""
        s, o = self.sys, self.out
        sa, sb = self.slot, self.slot_b
        main = main if main is not None else sa.stream
        side = sb.stream
        if serial:
            sb.set_stream(main)
            side = main
        nb = len(s.bodies)
        sids = [b["surf"] for b in s.bodies]
        cutters = s.bg_cutters()
        bufs = o["ib_bg"]
        ib_bg = bufs[k % len(bufs)]
        ident = self.poses_dev[self.n_pose - 1]
        if not serial and torch.cuda.is_current_stream_capturing():
            # one fork (and its join) per capture: the captured step is built
            # and tested in that form only
            if self._capture_forks:
                raise RuntimeError("SlotStep: a second stream fork inside one graph capture is not supported")
            self._capture_forks += 1
        side.wait_stream(main)
        # chain A: background
        if self.warm and not cold:
            sa.cut_warm(s.bg_id, cutters[0], self.poses_dev[0], self.sweep, bufs[(k - 1) % 2], ib_bg)
        else:
            sa.cut(s.bg_id, cutters, self.poses_dev[:nb], ib_bg)
        cap_bg = o["pts_bg"].shape[0]
        z = self.nodes1d
        if self.ab:
            sa.ab_faces(s.bg_id, ib_bg, o["faces_bg"], self.nf_dev[0:1])
            sa.face_points(s.bg_id, ident, o["faces_bg"], self.nf_dev[0:1], o["pts_bg"], self.n_dev[0:1], o["src_bg"],
                           nodes1d=z)
        else:
            sa.fringe_points(s.bg_id, ident, ib_bg, o["pts_bg"], self.n_dev[0:1], o["src_bg"])
        for i, b in enumerate(o["bodies"]):
            sa.donor_search(s.bodies[i]["shell"], self.poses_dev[i], o["pts_bg"], cap_bg, self.n_dev[0:1],
                            b["donor_bg"], b["ref_bg"])
            if self.ab:
                sa.interp_weights(b["donor_bg"], b["ref_bg"], cap_bg, self.n_dev[0:1], b["w_bg"], nodes1d=z)
        # chain B: shells
        r = nb
        for i, b in enumerate(s.bodies):
            others = [sids[j] for j in range(nb) if j != i]
            ob = o["bodies"][i]
            sb.cut_posed(b["shell"], self.poses_dev[i], others, self.poses_dev[r:r + nb - 1], ob["ib"])
            r += nb - 1
            cap = ob["pts"].shape[0]
            nd = self.n_dev[1 + i:2 + i]
            if self.ab:
                sb.ab_faces(b["shell"], ob["ib"], ob["faces"], self.nf_dev[1 + i:2 + i])
                sb.face_points(b["shell"], self.poses_dev[i], ob["faces"], self.nf_dev[1 + i:2 + i], ob["pts"], nd,
                               ob["src"], nodes1d=z)
            else:
                sb.fringe_points(b["shell"], self.poses_dev[i], ob["ib"], ob["pts"], nd, ob["src"])
            sb.donor_search(s.bg_id, ident, ob["pts"], cap, nd, ob["donor"], ob["ref"])
            if self.ab:
                sb.interp_weights(ob["donor"], ob["ref"], cap, nd, ob["w"], nodes1d=z)
        if serial:
            sb.set_stream(sb.stream)
        else:
            main.wait_stream(side)

    def set_poses(self, poses):
        with torch.cuda.stream(self.slot.stream):
            self.poses_dev.copy_(self._pose_table(poses))

    def _warm_ok(self, pose):
        """True when a warm cut from the last step's pose to ``pose`` (host,
        the body's) stays within the sweep bound the step was built with."""
        if self._last_pose is None:
            return True             # after a device table: the caller's bound
        need = self.sys.ctx.sweep_bound(self.sys.bg_cutters()[0], self._last_pose, pose)
        # sweep_bound is inflated by a relative 1e-9 beyond the true largest
        # travel, so equal steps whose bounds differ in the last bits still
        # pass, and a passing pose never moves a point farther than sweep
        return need <= self.sweep * (1.0 + 1e-9)

    def step(self, poses, cold=False, serial=False):
        """Eager launches on the slot streams (no synchronisation); the step
        is complete when the slot stream (``stream``) reaches its end.  The
        first step of a warm SlotStep (or one with ``cold``, or one whose
        pose moved farther than the sweep bound) is a cold cut; ``serial``
        runs both chains on the slot stream, one after the other."""
        if self.warm and self.k > 0 and not cold and not self._warm_ok(poses[0]):
            cold = True
            self.cold_fallbacks += 1
        self.set_poses(poses)
        self._launch(self.k, cold or self.k == 0, serial=serial)
        self.k += 1
        if self.warm:
            self._last_pose = np.asarray(poses[0], dtype=np.float64).copy()

    def capture(self):
        """Capture the step (both iblank parities when warm); a warm
        SlotStep must have run one eager step first."""
        if self.warm and self.k == 0:
            raise RuntimeError("run one eager step before capturing a warm step")
        torch.cuda.synchronize()
        side = self.slot_b.stream
        for par in ((0, 1) if self.warm else (0,)):
            g = torch.cuda.CUDAGraph()
            self._capture_forks = 0
            with torch.cuda.graph(g):
                cur = torch.cuda.current_stream()
                self.slot.set_stream(cur)
                self._launch(par, False, main=cur)
            self.slot.set_stream(self.slot.stream)
            self.slot_b.set_stream(side)
            self.graphs[par] = g
        return self.graphs

    def pose_table_dev(self, poses):
        """Device copy of the pose table of ``poses`` (for replay_table)."""
        return self._pose_table(poses).to(self.poses_dev.device)

    def replay(self, poses):
        """Graph replay of the next step on the slot stream with new poses."""
        self.replay_table(self._pose_table(poses))

    def replay_table(self, table):
        """Graph replay with a pose table (host, or device: then the copy is
        stream ordered and the host does not wait).  A warm step whose host
        table moves the body beyond the sweep bound runs eagerly and cold."""
        if not self.graphs:
            self.capture()
        if self.warm:
            if table.is_cuda:
                self._last_pose = None      # not read back: the caller keeps the bound
            else:
                pose = table[0].numpy().astype(np.float64)
                if not self._warm_ok(pose):
                    with torch.cuda.stream(self.slot.stream):
                        self.poses_dev.copy_(table)
                    self.cold_fallbacks += 1
                    self._launch(self.k, True)
                    self.k += 1
                    self._last_pose = pose.copy()
                    return
                self._last_pose = pose.copy()
        with torch.cuda.stream(self.slot.stream):
            self.poses_dev.copy_(table, non_blocking=table.is_cuda)
            self.graphs[self.k % 2 if self.warm else 0].replay()
        self.k += 1

    def counts(self):
        """Point counts (waits for the slot stream)."""
        self.slot.stream.synchronize()
        n = self.n_dev.cpu().tolist()
        out = dict(n_bg_points=n[0], n_shell_points=n[1:])
        if self.ab:
            f = self.nf_dev.cpu().tolist()
            out.update(n_bg_faces=f[0], n_shell_faces=f[1:])
        return out

    def snapshot(self):
        """Host copy of the last step's outputs (synchronises)."""
        c = self.counts()
        n_bg = c["n_bg_points"]
        o = self.out
        out = dict(ib_bg=self.ib_bg().cpu().numpy(), pts_bg=o["pts_bg"][:n_bg].cpu().numpy(),
                   src_bg=o["src_bg"][:n_bg].cpu().numpy(), bodies=[])
        nf = self.nf_dev.cpu().tolist()
        if self.ab:
            out["faces_bg"] = o["faces_bg"][:nf[0]].cpu().numpy()
        for i, (b, n) in enumerate(zip(o["bodies"], c["n_shell_points"])):
            d = dict(ib=b["ib"].cpu().numpy(), pts=b["pts"][:n].cpu().numpy(),
                     src=b["src"][:n].cpu().numpy(), donor_bg=b["donor_bg"][:n_bg].cpu().numpy(),
                     ref_bg=b["ref_bg"][:n_bg].cpu().numpy(), donor=b["donor"][:n].cpu().numpy(),
                     ref=b["ref"][:n].cpu().numpy())
            if self.ab:
                d.update(faces=b["faces"][:nf[1 + i]].cpu().numpy(), w=b["w"][:n].cpu().numpy(),
                         w_bg=b["w_bg"][:n_bg].cpu().numpy())
            out["bodies"].append(d)
        return out


class UnblankStep:
    """The time step of a moving body with unblanking (Sec. 3, Alg. unblank)
    on a slot of its own: the background cut at the poses of t and t + dt
    (wall rule), the cells to unblank, their 27 interior points and their
    donors in the body's near-body grid at t.  Poses and counts live on the
    device and nothing synchronises, so the step can be captured; the two
    iblank buffers alternate (step k reads buffer k mod 2 as the previous
    blanking and writes the other), so a captured step exists for each
    parity."""

    def __init__(self, ctx: _oc.Context, bg_id, surf_id, shell_id, ub_cap, stream=None):
        self.ctx = ctx
        self.bg, self.surf, self.shell = bg_id, surf_id, shell_id
        dev = torch.device("cuda", ctx.device)
        n_bg = ctx.grids[bg_id]
        # two cut instances per step (the wall at t and at t + dt)
        self.slot = ctx.create_slot([bg_id, shell_id], [surf_id, surf_id], 27 * ub_cap, stream)
        self.ib = [torch.empty(n_bg, dtype=torch.int8, device=dev) for _ in range(2)]
        self.ub = torch.empty(ub_cap, dtype=torch.int32, device=dev)
        self.n_ub = torch.zeros(1, dtype=torch.int32, device=dev)
        self.n_pts = torch.zeros(1, dtype=torch.int32, device=dev)
        cap = 27 * ub_cap
        self.cap = cap
        self.pts = torch.empty((cap, 3), dtype=torch.float64, device=dev)
        self.src = torch.empty(cap, dtype=torch.int32, device=dev)
        self.donor = torch.empty(cap, dtype=torch.int32, device=dev)
        self.ref = torch.empty((cap, 3), dtype=torch.float64, device=dev)
        # rows: pose at t, pose at t + dt, identity (the background's pose)
        self.poses = torch.zeros((3, 12), dtype=torch.float64, device=dev)
        self.k = 0
        self.graphs = {}

    @property
    def stream(self):
        return self.slot.stream

    def close(self):
        self.slot.close()

    def _table(self, pose_t, pose_tp):
        return torch.from_numpy(np.stack([np.asarray(pose_t, dtype=np.float64),
                                          np.asarray(pose_tp, dtype=np.float64), IDENTITY]))

    def start(self, pose0):
        """Plain cut at the first pose into the first iblank buffer."""
        with torch.cuda.stream(self.slot.stream):
            self.poses.copy_(self._table(pose0, pose0))
        self.slot.cut(self.bg, [self.surf], self.poses[0:1], self.ib[0])
        self.k = 0

    def _launch(self, k):
        s = self.slot
        prev, cur = self.ib[k % 2], self.ib[(k + 1) % 2]
        s.unblank(self.bg, [self.surf], self.poses[0:2], prev, cur, self.ub, self.n_ub)
        s.element_points(self.bg, self.poses[2], self.ub, self.n_ub, self.pts, self.n_pts, self.src)
        s.donor_search(self.shell, self.poses[0], self.pts, self.cap, self.n_pts, self.donor, self.ref)

    def step(self, pose_t, pose_tp):
        """Eager step k (no synchronisation)."""
        with torch.cuda.stream(self.slot.stream):
            self.poses.copy_(self._table(pose_t, pose_tp))
        self._launch(self.k)
        self.k += 1

    def capture(self):
        torch.cuda.synchronize()
        own = self.slot.stream
        for par in (0, 1):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.slot.set_stream(torch.cuda.current_stream())
                self._launch(par)
            self.slot.set_stream(own)
            self.graphs[par] = g
        return self.graphs

    def replay_table(self, table):
        """Graph replay of the next step with a device (or host) pose table
        [3, 12]: pose at t, at t + dt, identity."""
        if not self.graphs:
            self.capture()
        with torch.cuda.stream(self.slot.stream):
            self.poses.copy_(table, non_blocking=table.is_cuda)
            self.graphs[self.k % 2].replay()
        self.k += 1

    def replay(self, pose_t, pose_tp):
        self.replay_table(self._table(pose_t, pose_tp))

    def table_dev(self, pose_t, pose_tp):
        return self._table(pose_t, pose_tp).to(self.poses.device)

    def result(self):
        """Host copy of the last step (synchronises): new iblank, cells to
        unblank, their points and donors."""
        self.slot.stream.synchronize()
        n = int(self.n_ub.item())
        m = min(27 * n, self.cap)
        return dict(ib=self.ib[self.k % 2].cpu().numpy(), ub=self.ub[:n].cpu().numpy(),
                    pts=self.pts[:m].cpu().numpy(), src=self.src[:m].cpu().numpy(),
                    donor=self.donor[:m].cpu().numpy(), ref=self.ref[:m].cpu().numpy())
