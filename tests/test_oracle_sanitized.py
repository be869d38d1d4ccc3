"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
a checking build of oracle.c runs the oracle's entry points on small cases
(cut, lattice pins, donor search, fringe points, filtered cut, refined cut,
unblank) in a child process with the ASan runtime preloaded; any report
fails the test.  The child's results must also equal the normal build's."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, {root!r})
import os
import oracle as orc
from workloads import meshes as M
assert orc._LIB_PATH == (os.environ.get("ORACLE_LIB") or orc._LIB_PATH)
orc.lib()
rng = np.random.default_rng(3)
bg = M.background_grid(6, -1.0, 1.0, amp=0.04)
s = M.cube_sphere(3, R=0.45, dimples=6, dimple_a=0.08, dimple_k=0.03)
pose = M.random_pose(rng, 0.1)
out = {{}}
out["cut"] = orc.cut(bg, [s], [pose], threads=2)
out["cut_brute"] = orc.cut(bg, [s], [pose], brute=True, threads=1)
out["diag"] = orc.cut_surface(bg, s, pose, diagnostics=True)["dstar"]
A = rng.standard_normal((3, 3)); B = rng.standard_normal((3, 3))
out["tri"] = np.array([orc.tri_tri(A, B)[0]])
elems = np.nonzero(out["cut"] == orc.FRINGE)[0]
pts = orc.fringe_points(bg, elems, pose)
out["pts"] = pts
d, r = orc.donor_search(bg, pts[:200] * 0.9, threads=2)[:2]
out["donor"] = d
out["ref"] = np.nan_to_num(r)
out["heur"] = orc.cut_heuristic(bg, [s], [pose], nf1=8, nf2=2, threads=2)
out["refined"] = orc.cut_refined(bg, [s], [pose], 2, threads=2)
pose2 = pose.copy(); pose2[9] += 0.05
out["unblank"] = np.asarray(orc.unblank(bg, [s], [pose], [pose2], out["cut"], threads=2)[0])
np.savez(sys.argv[1], **out)
"""


def _run(tmp_path, name, env):
    script = tmp_path / ("child_%s.py" % name)
    script.write_text(CHILD.format(root=ROOT))
    res = tmp_path / ("res_%s.npz" % name)
    p = subprocess.run([sys.executable, str(script), str(res)], env=env, capture_output=True, text=True,
                       timeout=600)
    return p, res


def test_oracle_under_asan_and_ubsan(tmp_path):
    import numpy as np
    import oracle as orc
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not libasan or not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no ASan runtime here")
    lib = str(tmp_path / "liboracle_san.so")
    orc.build_sanitized(lib)
    env = dict(os.environ)
    env.update(ORACLE_LIB=lib, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    p, res = _run(tmp_path, "san", env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    plain_env = dict(os.environ)
    plain_env.pop("ORACLE_LIB", None)
    q, res_plain = _run(tmp_path, "plain", plain_env)
    assert q.returncode == 0, q.stderr[-4000:]
    a, b = np.load(res), np.load(res_plain)
    for k in b.files:
        assert np.array_equal(a[k], b[k]), k
