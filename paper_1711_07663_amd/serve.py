"""Serving loop: connectivity requests (a registered overset system and the
body poses of one time step) arrive over time and are served with continuous
batching on one device.

* Systems (grids, surfaces, donor bins) are registered once and stay on the
  device.
* Each in-flight request holds a slot: a SlotStep of its system with its own
  streams, scratch and outputs, whose step is a captured HIP graph.  A request
  is admitted as soon as an idle slot of its system exists, or a new slot fits
  in the HBM budget; otherwise it waits.  Admitted requests run concurrently
  on their slots' streams, so work of requests that arrive while others are
  on the device overlaps with theirs.
* Requests are taken in arrival order, except that a request whose system has
  no slot available does not hold back the requests behind it.

The loop is driven by the caller: submit() enqueues, pump() retires finished
requests (calling on_done while the slot still holds the outputs) and admits
waiting ones.  Latency of a request = retirement time - arrival time.
"""
from __future__ import annotations

import time
from collections import deque

import torch

from . import oc as _oc
from .pipeline import SlotStep


def _tensor_bytes(out):
    n = 0
    for v in out.values():
        if isinstance(v, torch.Tensor):
            n += v.numel() * v.element_size()
        elif isinstance(v, list):
            for x in v:
                n += _tensor_bytes(x) if isinstance(x, dict) else x.numel() * x.element_size()
    return n


class Server:
    def __init__(self, ctx: _oc.Context, systems, hbm_budget, max_slots=16, on_done=None, graphs=True):
        """systems: name -> OversetSystem (registered on ctx).  hbm_budget:
        device bytes that registered state plus all slots (scratch and
        outputs) may hold."""
        self.ctx = ctx
        self.systems = dict(systems)
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.on_done = on_done
        self.graphs = graphs
        self.idle = {k: [] for k in self.systems}
        self.slots = []
        self.queue = deque()
        self.busy = []
        self.done = []
        self.n_refused = 0
        # bytes of one slot of each system, measured on a slot made and
        # released here
        self.slot_size = {}
        for name, sysm in self.systems.items():
            ss = SlotStep(sysm)
            self.slot_size[name] = ss.nbytes() + _tensor_bytes(ss.out) + ss.poses_dev.numel() * 8
            ss.close()
            del ss

    def used_bytes(self):
        """Registered state and slot scratch (the library's count) plus the
        slots' output buffers."""
        return self.ctx.memory_used() + sum(_tensor_bytes(s.out) + s.poses_dev.numel() * 8 for s in self.slots)

    def _slot_for(self, name):
        if self.idle[name]:
            return self.idle[name].pop()
        if len(self.slots) >= self.max_slots:
            victim = next((k for k, v in self.idle.items() if k != name and v), None)
            if victim is None:
                return None
            self._release(self.idle[victim].pop())
        sysm = self.systems[name]
        est = self._estimate(name)
        # make room by releasing idle slots of other systems
        while self.used_bytes() + est > self.budget:
            victim = next((k for k, v in self.idle.items() if k != name and v), None)
            if victim is None:
                break
            self._release(self.idle[victim].pop())
        if self.used_bytes() + est > self.budget:
            self.n_refused += 1
            if not self.busy:
                raise RuntimeError("a request of system %r does not fit in the HBM budget" % name)
            return None
        try:
            ss = SlotStep(sysm)
        except _oc.OcError as e:
            if e.status == _oc.OC_EBUDGET:
                self.n_refused += 1
                return None
            raise
        self.slots.append(ss)
        return ss

    def _release(self, ss):
        ss.close()
        self.slots.remove(ss)
        ss.out = {}
        ss.graphs = {}

    def _estimate(self, name):
        return self.slot_size[name]

    def submit(self, system, poses, t_arrival=None, tag=None):
        req = dict(system=system, poses=[p for p in poses], t_arrival=time.perf_counter() if t_arrival is None
                   else t_arrival, tag=tag)
        self.queue.append(req)
        return req

    def pump(self):
        """Retire finished requests, admit waiting ones; returns the number
        of requests retired."""
        n_ret = 0
        still = []
        for req, ss, ev in self.busy:
            if ev.query():
                req["t_done"] = time.perf_counter()
                if self.on_done is not None:
                    self.on_done(req, ss)
                self.idle[req["system"]].append(ss)
                self.done.append(req)
                n_ret += 1
            else:
                still.append((req, ss, ev))
        self.busy = still
        blocked = set()
        i = 0
        while i < len(self.queue):
            req = self.queue[i]
            if req["system"] in blocked:
                i += 1
                continue
            ss = self._slot_for(req["system"])
            if ss is None:
                blocked.add(req["system"])
                i += 1
                continue
            del self.queue[i]
            req["t_start"] = time.perf_counter()
            if self.graphs:
                ss.replay(req["poses"])
            else:
                ss.step(req["poses"], cold=True)
            ev = torch.cuda.Event()
            ev.record(ss.stream)
            self.busy.append((req, ss, ev))
        return n_ret

    def drain(self):
        while self.queue or self.busy:
            self.pump()

    def in_flight(self):
        return len(self.busy)
