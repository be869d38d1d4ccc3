"""Helpers for comparing the HIP path with the oracle on the same seeded case."""
from __future__ import annotations

import numpy as np

import oracle as O

XI_TOL = 1e-10      # donor reference coordinates (FP64 path)
PT_TOL = 1e-12      # receptor point coordinates


def pose_inverse(p):
    R = np.asarray(p[:9]).reshape(3, 3)
    t = np.asarray(p[9:12])
    return np.concatenate([R.T.ravel(), -R.T @ t])


def pose_compose(a, b):
    Ra = np.asarray(a[:9]).reshape(3, 3)
    Rb = np.asarray(b[:9]).reshape(3, 3)
    return np.concatenate([(Ra @ Rb).ravel(), Ra @ np.asarray(b[9:12]) + np.asarray(a[9:12])])


def oracle_step(case, poses, threads=0):
    """The connectivity step computed by the oracle alone."""
    bg = case["bg"]
    walls = [b["surface"] for b in case["bodies"]]
    out = {}
    out["ib_bg"] = O.cut(bg, walls, poses, threads=threads)
    fe = O.fringe_elements(out["ib_bg"])
    out["pts_bg"] = O.fringe_points(bg, fe)
    out["src_bg"] = np.repeat(fe, 27)
    out["bodies"] = []
    for i, b in enumerate(case["bodies"]):
        others = [j for j in range(len(walls)) if j != i]
        inv = pose_inverse(poses[i])
        ib = O.cut(b["shell"], [walls[j] for j in others], [pose_compose(inv, poses[j]) for j in others],
                   threads=threads)
        fs = O.fringe_elements(ib)
        pts = O.fringe_points(b["shell"], fs, poses[i])
        d_bg, r_bg, _ = O.donor_search(b["shell"], out["pts_bg"], poses[i], threads=threads)
        d, r, _ = O.donor_search(bg, pts, threads=threads)
        out["bodies"].append(dict(ib=ib, pts=pts, src=np.repeat(fs, 27), donor_bg=d_bg, ref_bg=r_bg, donor=d, ref=r))
    return out


def element_boxes(grid, chunk=1 << 18):
    """Node boxes (lo, hi) of every element, computed in chunks."""
    n = grid.n_elem
    lo = np.empty((n, 3))
    hi = np.empty((n, 3))
    for d in range(3):
        x = np.ascontiguousarray(grid.nodes[:, d])
        for s in range(0, n, chunk):
            c = grid.conn[s:s + chunk]
            a = x[c[:, 0]]
            b = a.copy()
            for k in range(1, c.shape[1]):
                v = x[c[:, k]]
                np.minimum(a, v, out=a)
                np.maximum(b, v, out=b)
            lo[s:s + chunk, d] = a
            hi[s:s + chunk, d] = b
    return lo, hi


def band_hole_mask(grid, surfaces, poses, kinds=None, threads=0, pad=1e-4, boxes=None):
    """Holes of grid cut by posed surfaces, the oracle run only on the
    elements whose node box comes within pad of a posed surface's node box.
    Every other element is farther than pad (> 1e-7) from that surface and
    its first node lies outside the surface's box, hence outside the closed
    surface (winding number 0): not a hole under the plain definition."""
    if kinds is None:
        kinds = [O.SURF_WALL] * len(surfaces)
    lo, hi = boxes if boxes is not None else element_boxes(grid)
    hole = np.zeros(grid.n_elem, dtype=bool)
    n_band = 0
    for s, p, k in zip(surfaces, poses, kinds):
        R = np.asarray(p[:9], dtype=np.float64).reshape(3, 3)
        X = s.nodes @ R.T + np.asarray(p[9:12], dtype=np.float64)
        slo, shi = X.min(axis=0) - pad, X.max(axis=0) + pad
        band = np.nonzero(np.all(hi >= slo, axis=1) & np.all(lo <= shi, axis=1))[0]
        n_band += band.size
        if band.size:
            st = O.cut_surface(grid, s, p, k, sel=band, threads=threads)
            hole[band[st == 0]] = True
    return hole, n_band


def band_cut(grid, surfaces, poses, kinds=None, threads=0, boxes=None):
    """The oracle's iblank of a large grid by the band method (holes as
    band_hole_mask, then the fringe layer over the whole grid)."""
    hole, _ = band_hole_mask(grid, surfaces, poses, kinds, threads, boxes=boxes)
    return O.mark_fringe(hole, O.face_neighbors(grid.conn), grid.face_tags)


def oracle_step_band(case, poses, threads=0):
    """oracle_step for cases too large for a whole-grid oracle cut: the cuts
    by the band method, receptor points and donors for every point."""
    bg = case["bg"]
    walls = [b["surface"] for b in case["bodies"]]
    out = {}
    out["ib_bg"] = band_cut(bg, walls, poses, threads=threads)
    fe = O.fringe_elements(out["ib_bg"])
    out["pts_bg"] = O.fringe_points(bg, fe)
    out["src_bg"] = np.repeat(fe, 27)
    out["bodies"] = []
    for i, b in enumerate(case["bodies"]):
        others = [j for j in range(len(walls)) if j != i]
        inv = pose_inverse(poses[i])
        ib = band_cut(b["shell"], [walls[j] for j in others], [pose_compose(inv, poses[j]) for j in others],
                      threads=threads)
        fs = O.fringe_elements(ib)
        pts = O.fringe_points(b["shell"], fs, poses[i])
        d_bg, r_bg, _ = O.donor_search(b["shell"], out["pts_bg"], poses[i], threads=threads)
        d, r, _ = O.donor_search(bg, pts, threads=threads)
        out["bodies"].append(dict(ib=ib, pts=pts, src=np.repeat(fs, 27), donor_bg=d_bg, ref_bg=r_bg, donor=d, ref=r))
    return out


def gpu_step(system, poses):
    """The same step through the HIP library (pipeline.OversetSystem)."""
    import torch
    c = system.step(poses)
    torch.cuda.synchronize()
    n_bg = c["n_bg_points"]
    out = dict(ib_bg=system.ib_bg.cpu().numpy(), pts_bg=system.pts_bg[:n_bg].cpu().numpy(),
               src_bg=system.src_bg[:n_bg].cpu().numpy(), bodies=[])
    for b, n in zip(system.bodies, c["n_shell_points"]):
        out["bodies"].append(dict(ib=b["ib"].cpu().numpy(), pts=b["pts"][:n].cpu().numpy(),
                                  src=b["src"][:n].cpu().numpy(), donor_bg=b["donor_bg"][:n_bg].cpu().numpy(),
                                  ref_bg=b["ref_bg"][:n_bg].cpu().numpy(), donor=b["donor"][:n].cpu().numpy(),
                                  ref=b["ref"][:n].cpu().numpy()))
    return out


def _cmp_donors(d_g, r_g, d_o, r_o, what):
    assert d_g.shape == d_o.shape, what
    bad = np.nonzero(d_g != d_o)[0]
    assert bad.size == 0, "%s: %d donor ids differ, first %s: gpu %s oracle %s" % (
        what, bad.size, bad[:5], d_g[bad[:5]], d_o[bad[:5]])
    ok = d_o >= 0
    if ok.any():
        err = np.abs(r_g[ok] - r_o[ok]).max()
        assert err <= XI_TOL, "%s: max |xi_gpu - xi_oracle| = %g" % (what, err)
    assert np.all(np.isnan(r_g[~ok])), what + ": orphan reference coordinates must be NaN"


def compare(g, o):
    """Bit-exact iblank and donor ids, reference coordinates within XI_TOL."""
    bad = np.nonzero(g["ib_bg"] != o["ib_bg"])[0]
    assert bad.size == 0, "background iblank: %d elements differ, first %s: gpu %s oracle %s" % (
        bad.size, bad[:8], g["ib_bg"][bad[:8]], o["ib_bg"][bad[:8]])
    assert np.array_equal(g["src_bg"], o["src_bg"])
    if o["pts_bg"].size:
        assert np.abs(g["pts_bg"] - o["pts_bg"]).max() <= PT_TOL
    for k, (gb, ob) in enumerate(zip(g["bodies"], o["bodies"])):
        assert np.array_equal(gb["ib"], ob["ib"]), "shell %d iblank" % k
        assert np.array_equal(gb["src"], ob["src"])
        if ob["pts"].size:
            assert np.abs(gb["pts"] - ob["pts"]).max() <= PT_TOL
        # both directions searched from the oracle's own points would hide
        # point differences; the points agree to PT_TOL, so search results of
        # each side's own points are compared
        _cmp_donors(gb["donor_bg"], gb["ref_bg"], ob["donor_bg"], ob["ref_bg"], "bg->shell %d" % k)
        _cmp_donors(gb["donor"], gb["ref"], ob["donor"], ob["ref"], "shell %d->bg" % k)


def oracle_ab_step(case, poses, nodes1d=O.GAUSS3, threads=0, ib_bg=None, topology="walls"):
    """The artificial-boundary step computed by the oracle alone: AB faces of
    the background and of each shell, their flux points and donors (weights
    are compared at the GPU's own reference coordinates, see compare_ab).
    ib_bg: the background blanking when already known.  topology "paper":
    the background is cut by the shells' overset boundaries."""
    bg = case["bg"]
    walls = [b["surface"] for b in case["bodies"]]
    m2 = len(nodes1d) ** 2
    out = {}
    if ib_bg is None:
        if topology == "paper":
            ib_bg = O.cut(bg, [b["boundary"] for b in case["bodies"]], poses,
                          kinds=[O.SURF_OVERSET] * len(walls), threads=threads)
        else:
            ib_bg = O.cut(bg, walls, poses, threads=threads)
    out["ib_bg"] = ib_bg
    out["faces_bg"] = O.ab_faces(bg, out["ib_bg"])
    out["pts_bg"] = O.face_points(bg, out["faces_bg"], nodes1d)
    out["src_bg"] = np.repeat(out["faces_bg"], m2)
    out["bodies"] = []
    for i, b in enumerate(case["bodies"]):
        others = [j for j in range(len(walls)) if j != i]
        inv = pose_inverse(poses[i])
        ib = O.cut(b["shell"], [walls[j] for j in others], [pose_compose(inv, poses[j]) for j in others],
                   threads=threads)
        faces = O.ab_faces(b["shell"], ib)
        pts = O.face_points(b["shell"], faces, nodes1d, poses[i])
        d_bg, r_bg, _ = O.donor_search(b["shell"], out["pts_bg"], poses[i], threads=threads)
        d, r, _ = O.donor_search(bg, pts, threads=threads)
        out["bodies"].append(dict(ib=ib, faces=faces, pts=pts, src=np.repeat(faces, m2), donor_bg=d_bg,
                                  ref_bg=r_bg, donor=d, ref=r))
    return out


def _cmp_weights(w_g, donor, ref, nodes1d, what):
    w_o = O.interp_weights(donor, ref, nodes1d)
    assert w_g.shape == w_o.shape, what
    assert np.array_equal(np.isnan(w_g), np.isnan(w_o)), what
    ok = donor >= 0
    if ok.any():
        err = np.abs(w_g[ok] - w_o[ok]).max()
        assert err <= 1e-15, "%s: max |w_gpu - w_oracle| = %g" % (what, err)


def compare_ab(g, o, nodes1d=O.GAUSS3):
    """compare() plus bit-exact AB face lists and the weights, which the
    oracle evaluates at the GPU's reference coordinates (the same operations
    in the same order)."""
    compare(g, o)
    assert np.array_equal(g["faces_bg"], o["faces_bg"])
    for k, (gb, ob) in enumerate(zip(g["bodies"], o["bodies"])):
        assert np.array_equal(gb["faces"], ob["faces"]), "shell %d AB faces" % k
        _cmp_weights(gb["w_bg"], gb["donor_bg"], gb["ref_bg"], nodes1d, "bg->shell %d weights" % k)
        _cmp_weights(gb["w"], gb["donor"], gb["ref"], nodes1d, "shell %d->bg weights" % k)
