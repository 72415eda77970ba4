"""Continuous-batching FBP request server on one GPU.

Requests (volume shape, angles, detector, tilt, data) arrive over time.
Data may be device-resident or in pinned host memory; host data are copied
to the device on the request's slot stream, and with result_on_host the
volume is copied back into pinned host memory on the same stream, so the
measured latency then runs from arrival to the result on the host.

The server keeps a pool of execution slots; a slot owns a HIP stream
(default priority) and a workspace sized for one shape class.
A request is admitted as soon as a slot of its class is free or a new slot
fits in the HBM budget; its FBP is enqueued on the slot's stream at once,
so requests that arrive while others run overlap on the device.  Geometry
tables depend on the tilt, so each request gets its own host plan (cheap:
double-precision tables on the host); its table image is copied into the
slot's pinned staging buffer and uploaded asynchronously on the slot's
stream, and the plan is attached to the slot's device buffers without any
host synchronisation.  Plans of repeated (shape, tilt) pairs are cached.
The HBM budget counts every slot's tables and workspace plus, for each
running request, its output volume and the device copy of host data; a
request that could never fit is refused at submission.  Completion is
detected with an event per request; latency = completion - arrival.

Every result is the same whether a request runs alone or in a mix: the
operators are deterministic and a slot's workspace is private to it.
"""
import collections
import ctypes
import time

import numpy as np
import torch

from . import _abi
from .plan import Plan, _DTYPES, _FILTERS


class Request:
    __slots__ = ("rid", "shape", "tilt", "data", "arrival", "admitted", "done", "out", "out_host",
                 "event", "slot", "_dev_data")

    def __init__(self, rid, nz, n, n_theta, h, w, tilt, data, arrival=None):
        self.rid = rid
        self.shape = (nz, n, n_theta, h, w)
        self.tilt = float(tilt)
        self.data = data
        self.arrival = time.perf_counter() if arrival is None else arrival
        self.admitted = None
        self.done = None
        self.out = None
        self.out_host = None
        self.event = None
        self.slot = None
        self._dev_data = None

    @property
    def voxels(self):
        nz, n = self.shape[0], self.shape[1]
        return nz * n * n


class _Slot:
    def __init__(self, key, plan, device):
        self.key = key
        self.proto = plan           # plan whose buffers this slot owns
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.busy = None
        self.bytes = plan.tables.numel() + plan.work.numel()
        # pinned staging copy of a request's table image: rewritten only when
        # the slot is free, i.e. after the previous upload from it has run
        self.stage = torch.empty(plan.tables.numel(), dtype=torch.uint8, pin_memory=True)


class Server:
    """Admits FBP requests into per-class slots and runs them concurrently.

    max_slots bounds the number of concurrently running requests;
    hbm_budget bounds the device bytes of all slots (tables and workspaces)
    plus the outputs and device data copies of the running requests (0: no
    bound); a request larger than the budget on its own raises ValueError at
    submission;
    result_on_host copies every volume into pinned host memory (Request.out_host);
    keep_results=False drops a request's volumes once it has finished (a stream
    whose consumer only needs the timings keeps no outputs alive)."""

    def __init__(self, max_slots=4, hbm_budget=0, storage_dtype="f16", data_dtype="f32",
                 filter="shepp-logan", device=None, plan_cache=64, result_on_host=False,
                 keep_results=True):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.max_slots = max_slots
        self.hbm_budget = hbm_budget
        self.storage_dtype = storage_dtype
        self.data_dtype = data_dtype
        self.filter = filter
        self.result_on_host = result_on_host
        self.keep_results = keep_results
        self.slots = []
        self.queue = collections.deque()
        self.finished = []
        self._plans = collections.OrderedDict()
        self._plan_cache = plan_cache

    # ------------------------------------------------------------ plans
    def _class_key(self, req):
        return req.shape

    def _host_plan(self, req):
        """C-ABI plan handle for (shape, tilt); cached (host memory only)."""
        key = (req.shape, req.tilt)
        h = self._plans.get(key)
        if h is not None:
            self._plans.move_to_end(key)
            return h
        nz, n, nt, hh, w = req.shape
        g = _abi.lamino_geom()
        g.nz, g.n, g.n_theta, g.h, g.w, g.tilt = nz, n, nt, hh, w, req.tilt
        o = _abi.lamino_opts_default()
        o.data_dtype = _DTYPES[self.data_dtype][0]
        o.storage_dtype = _DTYPES[self.storage_dtype][0]
        o.filter = _FILTERS[self.filter]
        h = _abi.lamino_plan(g, o)
        self._plans[key] = h
        if len(self._plans) > self._plan_cache:
            _, old = self._plans.popitem(last=False)
            _abi.lamino_plan_destroy(old)
        return h

    def _slot_bytes(self, req):
        """Device bytes of a slot for the request's class (tables + workspace)."""
        t, w = _abi.lamino_plan_sizes(self._host_plan(req))
        return max(t, 256) + max(w, 256)

    @staticmethod
    def _request_bytes(req):
        """Device bytes a running request holds besides its slot: the output
        volume and, for host data, the device copy of the data."""
        nz, n = req.shape[0], req.shape[1]
        b = nz * n * n * 4
        if req.data.device.type == "cpu":
            b += req.data.numel() * req.data.element_size()
        return b

    def _used_bytes(self):
        return sum(s.bytes + (self._request_bytes(s.busy) if s.busy is not None else 0)
                   for s in self.slots)

    # ------------------------------------------------------------ admission
    def submit(self, req):
        if req.data.device.type == "cpu" and not req.data.is_pinned():
            raise ValueError(f"request {req.rid}: host data must be in pinned memory")
        if self.hbm_budget:
            need = self._slot_bytes(req) + self._request_bytes(req)
            if need > self.hbm_budget:
                raise ValueError(f"request {req.rid} needs {need} bytes of HBM, above the budget "
                                 f"of {self.hbm_budget}")
        self.queue.append(req)
        self._admit()

    def _free_slot(self, req):
        key = self._class_key(req)
        same = next((s for s in self.slots if s.busy is None and s.key == key), None)
        need = self._request_bytes(req) + (0 if same is not None else self._slot_bytes(req))
        # evict idle slots (other than the one to reuse) while the request does
        # not fit in the budget or no slot is available for a new one
        while (self.hbm_budget and self._used_bytes() + need > self.hbm_budget) or \
                (same is None and len(self.slots) >= self.max_slots):
            idle = [s for s in self.slots if s.busy is None and s is not same]
            if not idle:
                return None
            self.slots.remove(idle[0])
        if same is not None:
            return same
        nz, n, nt, h, w = req.shape
        proto = Plan(nz, n, nt, h, w, req.tilt, data_dtype=self.data_dtype,
                     storage_dtype=self.storage_dtype, filter=self.filter, device=self.device)
        slot = _Slot(key, proto, self.device)
        self.slots.append(slot)
        return slot

    def _admit(self):
        waiting = collections.deque()
        while self.queue:
            req = self.queue.popleft()
            slot = self._free_slot(req)
            if slot is None:
                waiting.append(req)
                continue
            self._launch(slot, req)
        self.queue = waiting

    def _launch(self, slot, req):
        h = self._host_plan(req)
        proto = slot.proto
        stream = slot.stream
        # the request's tables go into the slot's device buffer by an
        # asynchronous upload on the slot's stream; attaching the plan to the
        # slot's buffers involves no HIP call, so nothing here blocks the host
        _abi.lamino_plan_table_image(h, ctypes.c_void_p(slot.stage.data_ptr()), slot.stage.numel())
        nz, n = req.shape[0], req.shape[1]
        with torch.cuda.stream(stream):
            proto.tables.copy_(slot.stage, non_blocking=True)
        _abi.lamino_plan_attach(h, ctypes.c_void_p(proto.tables.data_ptr()),
                                ctypes.c_void_p(proto.work.data_ptr()))
        with torch.cuda.stream(stream):
            if req.data.device.type == "cpu":  # pinned (checked at submission)
                req._dev_data = req.data.to(self.device, non_blocking=True)
            else:
                req._dev_data = req.data
                req.data.record_stream(stream)
            req.out = torch.empty((nz, n, n), dtype=torch.float32, device=self.device)
        _abi.lamino_fbp(h, ctypes.c_void_p(req._dev_data.data_ptr()), ctypes.c_void_p(req.out.data_ptr()),
                        ctypes.c_void_p(stream.cuda_stream))
        if self.result_on_host:
            req.out_host = torch.empty((nz, n, n), dtype=torch.float32, pin_memory=True)
            with torch.cuda.stream(stream):
                req.out_host.copy_(req.out, non_blocking=True)
        req.event = torch.cuda.Event()
        req.event.record(stream)
        req.admitted = time.perf_counter()
        req.slot = slot
        slot.busy = req

    # ------------------------------------------------------------ progress
    def poll(self):
        """Retire finished requests, admit waiting ones; returns #finished."""
        n = 0
        for s in self.slots:
            r = s.busy
            if r is not None and r.event.query():
                r.done = time.perf_counter()
                r._dev_data = None
                if not self.keep_results:
                    r.out = r.out_host = None
                s.busy = None
                self.finished.append(r)
                n += 1
        if n or self.queue:
            self._admit()
        return n

    def drain(self):
        while self.queue or any(s.busy is not None for s in self.slots):
            if not self.poll():
                time.sleep(2e-5)

    def close(self):
        self.drain()
        for h in self._plans.values():
            _abi.lamino_plan_destroy(h)
        self._plans.clear()
        self.slots.clear()

    # ------------------------------------------------------------ metrics
    def stats(self):
        lat = np.array([r.done - r.arrival for r in self.finished]) * 1e3
        if len(lat) == 0:
            return {}
        t0 = min(r.arrival for r in self.finished)
        t1 = max(r.done for r in self.finished)
        vox = sum(r.voxels for r in self.finished)
        return {"requests": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "throughput_rps": len(lat) / (t1 - t0), "gvoxel_per_s": vox / (t1 - t0) / 1e9}


def run_poisson(server, classes, rate, count, seed=0, tilt_range=(20.0, 40.0)):
    """Submit `count` requests with Poisson arrivals at `rate` per second.

    classes: list of (nz, n, n_theta, h, w, data); each request draws a class
    uniformly.  data is either one tensor, used at a tilt drawn uniformly in
    tilt_range (degrees), or a dict {tilt in degrees: tensor} of data
    projected at each tilt, from which the request draws a tilt uniformly."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    picks = rng.integers(0, len(classes), size=count)
    uni = rng.uniform(*tilt_range, size=count)
    which = rng.random(size=count)
    start = time.perf_counter()
    arrivals = start + np.cumsum(gaps)
    for i in range(count):
        while time.perf_counter() < arrivals[i]:
            server.poll()
        nz, n, nt, h, w, data = classes[picks[i]]
        if isinstance(data, dict):
            keys = sorted(data)
            deg = keys[min(int(which[i] * len(keys)), len(keys) - 1)]
            d = data[deg]
        else:
            deg, d = uni[i], data
        server.submit(Request(i, nz, n, nt, h, w, np.deg2rad(deg), d, arrival=float(arrivals[i])))
    server.drain()
    return server.stats()
