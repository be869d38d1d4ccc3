"""The FP32 candidate filter's rounding bound (R12 reading of the box filter:
every box rounded outward to FP32, face boxes inflated by
delta = 1e-7 + 2^-20 max|x| before rounding).

The filter may keep extra pairs but must keep every (element, face) pair
whose exact distance is below the 1e-7 hit threshold.  Such a pair's FP64
node boxes are within 1e-7 of each other on every axis, so it suffices that
every pair with FP64 box gaps <= 1e-7 passes the FP32 test.  This checks
that statement of the rule, with the rule written out here in numpy as the
library states it (outward rounding by one FP32 step where the nearest FP32
value lies on the wrong side), on the tiny case, a 40^3 dimpled case and a
copy of the tiny case moved to |x| ~ 1e3, where the 2^-20 max|x| term is
what keeps the bound (1e-7 is far below an FP32 step there).  The HIP
kernels' own filter is checked through parity at the same sizes and
offsets (test_gpu_configs.py)."""
import numpy as np
import pytest

import parity_util as PU
from workloads import configs as CF
from workloads import meshes as M

TOL_HIT = 1e-7


def f32_down(v):
    f = v.astype(np.float32)
    bad = f.astype(np.float64) > v
    f[bad] = np.nextafter(f[bad], np.float32(-np.inf))
    return f


def f32_up(v):
    f = v.astype(np.float32)
    bad = f.astype(np.float64) < v
    f[bad] = np.nextafter(f[bad], np.float32(np.inf))
    return f


def fp32_boxes(elo, ehi, flo, fhi, fmaxabs):
    delta = TOL_HIT + np.ldexp(fmaxabs, -20)
    return f32_down(elo), f32_up(ehi), f32_down(flo - delta[:, None]), f32_up(fhi + delta[:, None])


def _pairs_within(elo, ehi, flo, fhi, gap):
    """(element, face) pairs whose FP64 boxes are within gap on every axis."""
    from scipy.spatial import cKDTree
    ec, er = 0.5 * (elo + ehi), 0.5 * np.linalg.norm(ehi - elo, axis=1)
    fc, fr = 0.5 * (flo + fhi), 0.5 * np.linalg.norm(fhi - flo, axis=1)
    cand = cKDTree(fc).query_ball_point(ec, er + fr.max() + 2 * gap)
    cnt = np.fromiter((len(c) for c in cand), dtype=np.int64, count=len(cand))
    ei = np.repeat(np.arange(elo.shape[0]), cnt)
    fi = np.fromiter((f for c in cand for f in c), dtype=np.int64, count=int(cnt.sum()))
    ok = np.all(fhi[fi] >= elo[ei] - gap, axis=1) & np.all(flo[fi] <= ehi[ei] + gap, axis=1)
    return ei[ok], fi[ok], ei.size


def _case(name):
    if name == "tiny":
        c = CF.tiny()
        return c["bg"], c["bodies"][0]["surface"], M.IDENTITY_POSE
    if name == "dimpled40":
        c = CF.dimpled(bg_n=40, m=16, layers=2, dimples=60)
        return c["bg"], c["bodies"][0]["surface"], M.pose_rz(0.3, (0.01, -0.02, 0.03))
    if name == "far":
        return far_tiny()
    raise KeyError(name)


def far_tiny():
    """The tiny case moved to about (1000, 1000, 1000): background 16^3 on
    [998, 1002]^3 (the sinusoid displaces its nodes as anywhere else), the
    96-face sphere posed there."""
    c = CF.tiny()
    bg = M.background_grid(16, 998.0, 1002.0, amp=0.02)
    return bg, c["bodies"][0]["surface"], np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 1000.0, 1000.0, 1000.0])


@pytest.mark.parametrize("name", ["tiny", "dimpled40", "far"])
def test_fp32_filter_keeps_every_close_pair(name):
    bg, s, pose = _case(name)
    elo, ehi = PU.element_boxes(bg)
    R = np.asarray(pose[:9]).reshape(3, 3)
    X = (s.nodes @ R.T + np.asarray(pose[9:12]))[s.conn]
    flo, fhi = X.min(axis=1), X.max(axis=1)
    fmaxabs = np.abs(X).max(axis=(1, 2))
    ei, fi, n_cand = _pairs_within(elo, ehi, flo, fhi, TOL_HIT)
    assert ei.size > 50
    a_lo, a_hi, b_lo, b_hi = fp32_boxes(elo, ehi, flo, fhi, fmaxabs)
    keep = np.all(a_hi[ei] >= b_lo[fi], axis=1) & np.all(a_lo[ei] <= b_hi[fi], axis=1)
    assert keep.all(), "%s: %d close pairs dropped by the FP32 filter" % (name, (~keep).sum())
