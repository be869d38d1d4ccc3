"""Host-side logic that needs no GPU: the serving loop's admission and
retirement (with a stand-in step), the batch autotuner's size classes, the
benchmark's traffic bookkeeping and argument checks, and the batch
generator."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


# ------------------------------------------------------------ serving loop --
class _FakeEvent:
    clock = [0]

    def __init__(self):
        self.t = None

    def record(self, stream):
        self.t = stream.busy_until

    def query(self):
        return _FakeEvent.clock[0] >= self.t


class _FakeStream:
    def __init__(self):
        self.busy_until = 0


class _NoBytes:
    def numel(self):
        return 0


class _FakeSlotStep:
    """Stands in for pipeline.SlotStep: a request occupies the slot for
    ``cost`` ticks of the fake clock."""
    made = []
    size = {}

    def __init__(self, system):
        self.sys = system
        self.stream = _FakeStream()
        self.out = {}
        self.poses_dev = _NoBytes()
        self.closed = False
        self.ran = []
        _FakeSlotStep.made.append(self)

    def nbytes(self):
        return self.size[self.sys["name"]]

    def close(self):
        self.closed = True

    def replay(self, poses):
        self.ran.append(poses)
        self.stream.busy_until = _FakeEvent.clock[0] + self.sys["cost"]

    def step(self, poses, cold=False):
        self.replay(poses)


class _FakeCtx:
    """The library counts every slot's scratch in memory_used()."""
    def __init__(self, base):
        self.base = base

    def memory_used(self):
        return self.base + sum(s.nbytes() for s in _FakeSlotStep.made if not s.closed)


@pytest.fixture
def fake_server(monkeypatch):
    torch = pytest.importorskip("torch")
    from paper_1711_07663_amd import serve
    monkeypatch.setattr(serve, "SlotStep", _FakeSlotStep)
    monkeypatch.setattr(torch.cuda, "Event", _FakeEvent)
    monkeypatch.setattr(serve, "_tensor_bytes", lambda out: 0)
    _FakeSlotStep.made = []
    _FakeEvent.clock[0] = 0

    def make(budget, sizes, costs, max_slots=16):
        _FakeSlotStep.size = dict(sizes)
        systems = {k: dict(name=k, cost=costs[k]) for k in sizes}
        done = []
        srv = serve.Server(_FakeCtx(100), systems, budget, max_slots=max_slots,
                           on_done=lambda req, ss: done.append((req["tag"], ss)))
        return srv, done
    return make


def _run(srv, ticks):
    for _ in range(ticks):
        srv.pump()
        _FakeEvent.clock[0] += 1


def test_serve_admits_concurrently_and_retires(fake_server):
    srv, done = fake_server(budget=10_000, sizes=dict(a=100, b=200), costs=dict(a=3, b=5))
    for i in range(6):
        srv.submit("a" if i % 2 == 0 else "b", [i], tag=i)
    srv.pump()
    # every request got its own slot at once (budget and slot count allow)
    assert srv.in_flight() == 6 and not srv.queue
    _run(srv, 10)
    assert sorted(t for t, _ in done) == list(range(6))
    # slots are reused by later requests instead of new ones being made
    made = len(_FakeSlotStep.made)
    srv.submit("a", [9], tag=9)
    _run(srv, 5)
    assert len(_FakeSlotStep.made) == made and 9 in [t for t, _ in done]


def test_serve_budget_waits_and_evicts(fake_server):
    # room for one slot of either system beside the registered state
    srv, done = fake_server(budget=100 + 250, sizes=dict(a=200, b=250), costs=dict(a=2, b=2))
    for i in range(4):
        srv.submit("a" if i < 2 else "b", [i], tag=i)
    srv.pump()
    assert srv.in_flight() == 1          # only one slot fits
    assert srv.n_refused > 0
    _run(srv, 20)
    assert sorted(t for t, _ in done) == [0, 1, 2, 3]
    # the idle slot of "a" was released to make room for "b"
    assert any(s.closed and s.sys["name"] == "a" for s in _FakeSlotStep.made)
    assert all(s.nbytes() <= 250 for s in srv.slots)


def test_serve_blocked_system_does_not_hold_back_others(fake_server):
    srv, done = fake_server(budget=100 + 300, sizes=dict(a=200, b=100), costs=dict(a=50, b=1), max_slots=2)
    srv.submit("a", [0], tag=0)
    srv.pump()
    srv.submit("a", [1], tag=1)     # waits: a second "a" slot does not fit
    srv.submit("b", [2], tag=2)     # fits beside the busy "a" slot
    srv.pump()
    assert srv.in_flight() == 2 and [r["tag"] for r in srv.queue] == [1]
    _run(srv, 5)
    assert [t for t, _ in done] == [2]
    _run(srv, 200)
    assert sorted(t for t, _ in done) == [0, 1, 2]


def test_serve_request_that_never_fits_raises(fake_server):
    srv, done = fake_server(budget=100 + 50, sizes=dict(a=200), costs=dict(a=1))
    srv.submit("a", [0], tag=0)
    with pytest.raises(RuntimeError):
        srv.pump()


# ---------------------------------------------------------------- autotune --
def test_autotune_size_classes():
    pytest.importorskip("torch")
    from paper_1711_07663_amd import autotune
    assert autotune.size_class(384) == 8
    assert autotune.size_class(24576) == 14
    assert autotune.size_class(1) == 0
    assert [autotune.size_class(6 * m * m) for m in (8, 16, 32, 64)] == [8, 10, 12, 14]


def test_autotune_file_round_trip(tmp_path):
    pytest.importorskip("torch")
    from paper_1711_07663_amd import autotune
    params = dict(exact_waves=4096, filter_block=512, bin_factor={"8": 0.75, "14": 0.5, "10": 1.0})
    path = str(tmp_path / "t.txt")
    autotune.save(params, path)
    text = open(path).read()
    assert "filter_block 512" in text and "bin_factor 14 0.5" in text
    assert autotune.load(path) == params


# ------------------------------------------------------------------- bench --
def test_bench_traffic_follows_kernel_source(tmp_path, monkeypatch):
    import bench
    for k in ("k_dp_newton", "k_filter"):
        assert bench.kernel_source_sha(k) is not None
        t = bench.measured_traffic(k)
        assert t is None or t > 1e6
    # an edited comment or spacing leaves the code, and the stored traffic, as
    # they were; a changed definition makes the stored traffic stale
    text = open(os.path.join(ROOT, bench.KERNEL_SOURCE["k_filter"])).read()
    assert "// a3, streaming part" in text and "int flags = 0, cn = 0;" in text
    t0 = bench.measured_traffic("k_filter")
    src = tmp_path / "k.hip"
    src.write_text(text.replace("// a3, streaming part", "// a3 (edited), streaming part", 1)
                   .replace("int flags = 0, cn = 0;", "int flags = 0,  cn = 0;", 1))
    monkeypatch.setitem(bench.KERNEL_SOURCE, "k_filter", str(src))
    assert bench.measured_traffic("k_filter") == t0
    src2 = tmp_path / "k2.hip"
    src2.write_text(text.replace("int flags = 0, cn = 0;", "int flags = 0, cn = 1;", 1))
    monkeypatch.setitem(bench.KERNEL_SOURCE, "k_filter", str(src2))
    assert bench.measured_traffic("k_filter") is None
    # so does a change to a device function in a shared header
    hdr = tmp_path / "q2.h"
    hdr.write_text(open(os.path.join(ROOT, "paper_1711_07663_amd/csrc/q2.h")).read() + "\n#define OC_EDITED 1\n")
    monkeypatch.setattr(bench, "KERNEL_HEADERS", [str(hdr) if h.endswith("q2.h") else h for h in bench.KERNEL_HEADERS])
    assert bench.measured_traffic("k_dp_newton") is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


# --------------------------------------------------------------- workloads --
def test_batch_instances_recipe():
    from workloads import configs as CF
    a = CF.batch_instances()
    b = CF.batch_instances()
    assert len(a) == 64
    assert [x["bg_n"] for x in a] == [x["bg_n"] for x in b]          # seeded
    assert all(16 <= x["bg_n"] <= 96 and 8 <= x["m"] <= 64 for x in a)
    kinds = {x["kind"] for x in a}
    assert kinds == {"sphere", "ellipsoid", "dimpled"}
    assert all((x["dimples"] == 0) == (x["kind"] != "dimpled") for x in a)
    assert all(50 <= x["dimples"] <= 300 for x in a if x["kind"] == "dimpled")
    for x in a:
        R = np.asarray(x["pose"][:9]).reshape(3, 3)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and np.linalg.det(R) > 0
        assert np.all(np.abs(x["pose"][9:]) <= 0.3)
