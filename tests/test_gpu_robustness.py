"""The HIP cut against the oracle on the connectivity-robustness cases of
Sec. 4.4 (a slot through the body, a narrow groove with high-aspect faces,
rotated and anisotropic backgrounds) and on a blade built so that the tie
rule of Sec. 4.1 (Fig. multinorm) averages opposite-sign normals; donor
search on the rotated anisotropic background.  Bar: iblank and donor ids
bit-exact, reference coordinates within 1e-10."""
import sys

import numpy as np
import pytest

import robust_cases as RC

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1711_07663_amd import oc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = oc.Context(device=0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("name", RC.NAMES)
def test_robustness_cut_parity(ctx, orc, name):
    import torch
    _note("robustness case %s: cut" % name)
    bg, s, pose = RC.case(name)
    gid = ctx.register_grid(bg.nodes, bg.conn)
    sid = ctx.register_cut_surface(s.nodes, s.conn)
    ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
    ctx.cut(gid, sid, pose, ib)
    info = ctx.last_cut_info()
    got = ib.cpu().numpy()
    want = orc.cut(bg, [s], [pose])
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s: %d elements differ, first %s: gpu %s oracle %s" % (
        name, bad.size, bad[:8], got[bad[:8]], want[bad[:8]])
    assert info["n_side"] > 0, "the nearest-face side search must run on this case"
    if name == "wedge":
        assert got[RC.WEDGE_ELEMENT] != orc.HOLE


def test_rotated_anisotropic_donors(ctx, orc):
    import torch
    _note("donor search in the rotated anisotropic background")
    bg, _, _ = RC.case("slot3d")
    gid = ctx.register_grid(bg.nodes, bg.conn)
    rng = np.random.default_rng(4403)
    pts = rng.uniform(-1.7, 1.7, size=(20000, 3))
    pose = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0.01, -0.02, 0.005])
    n = pts.shape[0]
    p = torch.from_numpy(pts).cuda()
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    r = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    ctx.donor_search(gid, pose, p, n, d, r)
    torch.cuda.synchronize()
    d_g, r_g = d.cpu().numpy(), r.cpu().numpy()
    d_o, r_o, _ = orc.donor_search(bg, pts, pose)
    assert np.array_equal(d_g, d_o)
    ok = d_o >= 0
    assert ok.sum() > 1000 and (~ok).sum() > 100
    assert np.abs(r_g[ok] - r_o[ok]).max() <= 1e-10
    assert np.all(np.isnan(r_g[~ok]))
