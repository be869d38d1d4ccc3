"""The bounds-checked build (liboc_checked.so, compiled with OC_CHECKED):
the small parity cases, a batch, a refined cut and a donor search forced
through its pair-overflow path run in a child process on that library; their
results match the oracle and the check word stays zero (no bin range,
record, pair or element index out of its array).  The product library
reports itself unchecked with a zero word."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import numpy as np
import torch
import oracle as orc
from paper_1711_07663_amd import oc
from paper_1711_07663_amd.pipeline import OversetSystem
from workloads import configs as CF
from workloads import meshes as M
import parity_util as PU
out = {{}}
ctx = oc.Context(device=0)
print("[checked] tiny step", flush=True)
case = CF.tiny()
system = OversetSystem(ctx, case)
g = PU.gpu_step(system, case["poses"])
PU.compare(g, PU.oracle_step(case, case["poses"]))
print("[checked] small batch", flush=True)
specs = CF.batch_instances(n=6, n_lo=8, n_hi=20, m_lo=3, m_hi=8)
cases = [CF.batch_case(s, layers=2) for s in specs]
reqs, want = [], []
for c in cases:
    gid = ctx.register_grid(c["bg"].nodes, c["bg"].conn)
    sid = ctx.register_cut_surface(c["bodies"][0]["surface"].nodes, c["bodies"][0]["surface"].conn)
    ib = torch.empty(c["bg"].n_elem, dtype=torch.int8, device="cuda")
    reqs.append((gid, [sid], c["poses"][0].reshape(1, 12), ib))
    want.append(orc.cut(c["bg"], [c["bodies"][0]["surface"]], [c["poses"][0]]))
ctx.cut_batch(reqs)
torch.cuda.synchronize()
for r, w in zip(reqs, want):
    assert np.array_equal(r[3].cpu().numpy(), w)
print("[checked] refined cut", flush=True)
rng = np.random.default_rng(7)
bg = M.background_grid(12, -1.0, 1.0, amp=0.05)
s = M.cube_sphere(4, R=0.5, dimples=12, dimple_a=0.1, dimple_k=0.03)
pose = M.random_pose(rng, 0.1)
gid = ctx.register_grid(bg.nodes, bg.conn)
sid = ctx.register_cut_surface(s.nodes, s.conn)
ib = torch.empty(bg.n_elem, dtype=torch.int8, device="cuda")
ctx.cut_refined(gid, [sid], pose[None], ib, 2)
assert np.array_equal(ib.cpu().numpy(), orc.cut_refined(bg, [s], [pose], 2))
print("[checked] donor search through the pair-overflow path", flush=True)
pts = rng.uniform(-0.9, 0.9, size=(3000, 3))
ctx.tune(oc.OC_TUNE_DONOR_PAIRS, 0, 500)
d = torch.empty(3000, dtype=torch.int32, device="cuda")
x = torch.empty((3000, 3), dtype=torch.float64, device="cuda")
ctx.donor_search(gid, M.IDENTITY_POSE, torch.from_numpy(pts).cuda(), 3000, d, x)
info = ctx.last_donor_info()
dw, xw = orc.donor_search(bg, pts)[:2]
assert np.array_equal(d.cpu().numpy(), dw)
ok = dw >= 0
assert np.abs(x.cpu().numpy()[ok] - xw[ok]).max() < 1e-10
assert info["n_overflow"] > 0
ctx.tune(oc.OC_TUNE_DONOR_PAIRS, 0, 0)
word, checked = ctx.check_word()
out.update(word=word, checked=checked)
ctx.close()
print(json.dumps(out), flush=True)
"""


def test_checked_build_runs_clean(tmp_path):
    from paper_1711_07663_amd import oc
    lib = os.path.join(ROOT, "paper_1711_07663_amd", "liboc_checked.so")
    assert os.path.exists(lib), "liboc_checked.so is built with the product library"
    script = tmp_path / "child.py"
    script.write_text(CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests")))
    env = dict(os.environ, OC_LIB=lib)
    p = subprocess.run([sys.executable, "-u", str(script)], env=env, capture_output=True, text=True, timeout=600)
    print(p.stdout[-2000:])
    assert p.returncode == 0, p.stderr[-4000:]
    res = json.loads(p.stdout.strip().splitlines()[-1])
    assert res["checked"] is True
    assert res["word"] == 0, "bounds check word %#x" % res["word"]


def test_product_build_reports_unchecked():
    import torch
    from paper_1711_07663_amd import oc
    assert torch.cuda.is_available()
    ctx = oc.Context(device=0)
    try:
        word, checked = ctx.check_word(clear=True)
        assert checked is False and word == 0
    finally:
        ctx.close()
