"""Continuous-batching request loop for many simulated camera streams.

Frames arrive per camera stream; a frame is admitted to one of ``n_slots`` worker slots
as soon as a slot is free and its stream's device state fits the HBM budget. Each
stream keeps its state resident on the device between frames (solver workspace,
output maps, input buffers), so a stream's frames reuse it; idle streams are evicted
least-recently-used when a new stream needs room. Frames of one stream are solved in
arrival order, one at a time; frames of different streams overlap on the device (each
slot has its own HIP stream and host thread, and the solver releases the GIL).

``Admission`` is the host-side policy alone (no GPU): it is driven by the server, and
by the CPU tests with a simulated clock and a fake budget. ``StereoServer`` executes
admitted frames with the library's ``sm_solve``; every step of the method runs in the
library.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple


@dataclass
class Request:
    rid: int
    stream: int
    t_arrival: float
    payload: object = None          # (left, right) host arrays or device tensors
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    status: int = 0
    result: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Admission:
    """FIFO admission under a device-memory budget with resident per-stream state.

    ``state_bytes(stream)`` gives the bytes a stream needs while resident. A request is
    admissible when its stream is not busy and either its state is resident or can be
    made resident by allocating (budget permitting) after evicting idle resident
    streams in least-recently-used order. Requests are considered in arrival order; a
    request that cannot be admitted does not block later requests of other streams
    whose state is already resident (no head-of-line blocking on memory)."""

    def __init__(self, budget_bytes: int, state_bytes: Callable[[int], int]):
        self.budget = int(budget_bytes)
        self.state_bytes = state_bytes
        self.used = 0
        self.resident: "collections.OrderedDict[int, int]" = collections.OrderedDict()  # LRU
        self.busy: set = set()
        self.queue: List[Request] = []
        self.evictions = 0

    def push(self, req: Request):
        need = self.state_bytes(req.stream)
        if need > self.budget:
            raise ValueError(f"stream {req.stream} needs {need} bytes, budget is {self.budget}")
        self.queue.append(req)

    def _make_room(self, need: int) -> Optional[List[int]]:
        if self.used + need <= self.budget:
            return []
        victims, freed = [], 0
        for s, b in self.resident.items():          # oldest first
            if s in self.busy:
                continue
            victims.append(s)
            freed += b
            if self.used - freed + need <= self.budget:
                return victims
        return None

    def next(self) -> Optional[Tuple[Request, List[int]]]:
        """Pops the next admissible request; returns it with the streams to evict."""
        for i, r in enumerate(self.queue):
            if r.stream in self.busy:
                continue
            if any(q.stream == r.stream for q in self.queue[:i]):
                continue                            # keep each stream's frames in order
            if r.stream in self.resident:
                victims = []
            else:
                victims = self._make_room(self.state_bytes(r.stream))
                if victims is None:
                    continue
            for s in victims:
                self.used -= self.resident.pop(s)
                self.evictions += 1
            if r.stream not in self.resident:
                b = self.state_bytes(r.stream)
                self.resident[r.stream] = b
                self.used += b
            self.resident.move_to_end(r.stream)
            self.busy.add(r.stream)
            del self.queue[i]
            return r, victims
        return None

    def done(self, req: Request):
        self.busy.discard(req.stream)


@dataclass
class StreamSpec:
    W: int
    H: int
    params: dict


class StereoServer:
    """Executes admitted frames on ``n_slots`` worker slots (thread + HIP stream each).

    ``specs[stream]`` gives each camera stream's frame size and method parameters.
    ``on_done(req, D_f, C_f, mask)`` is called on the worker thread after the frame's
    outputs are complete (device tensors of the stream's resident state, valid until
    that stream's next frame). ``device_mesh`` True (the default) keeps every
    tessellation on the GPU; each is one long single-workgroup kernel, so with many more
    slots than the device's hardware queues they wait on each other, and False
    (triangulation on the host, overlapped with other frames' kernels) can serve more
    frames per second there."""

    def __init__(self, specs: Dict[int, StreamSpec], n_slots: int, budget_bytes: int,
                 device="cuda:0", on_done=None, device_mesh: bool = True):
        import torch
        from . import api
        self._torch = torch
        self._api = api
        specs = {s: StreamSpec(sp.W, sp.H, dict(sp.params, host_mesh=0 if device_mesh else 1))
                 for s, sp in specs.items()}
        self.specs = specs
        self.device = device
        self.on_done = on_done
        self.lib = api._lib.load()
        self._ws_need = {}
        for s, sp in specs.items():
            self._ws_need[s] = self.lib.sm_solve_workspace_bytes(sp.W, sp.H, api.make_params(sp.params))
        self.adm = Admission(budget_bytes, self.state_bytes)
        self.n_slots = n_slots
        self.cv = threading.Condition()
        self.free_slots = list(range(n_slots))
        self.slot_streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]
        self.state: Dict[int, dict] = {}
        self.completed: List[Request] = []
        self.closed = False
        self._stop = False
        self.errors: List[str] = []
        self._rid = 0
        # one persistent thread per slot (the solver keeps per-thread host state)
        self._slot_req: List[Optional[Request]] = [None] * n_slots
        self._threads = [threading.Thread(target=self._slot_loop, args=(k,), daemon=True)
                         for k in range(n_slots)]
        for t in self._threads:
            t.start()
        self._dispatch = threading.Thread(target=self._dispatcher, daemon=True)
        self._dispatch.start()

    # --- memory accounting -----------------------------------------------------------
    def state_bytes(self, stream: int) -> int:
        sp = self.specs[stream]
        return int(self._ws_need[stream]) + sp.W * sp.H * (4 + 1 + 1 + 2)

    def _ensure_state(self, stream: int, cuda_stream):
        st = self.state.get(stream)
        if st is None:
            torch = self._torch
            sp = self.specs[stream]
            with torch.cuda.stream(cuda_stream):
                solver = self._api.Solver(sp.W, sp.H, sp.params, device=self.device)
                st = {"solver": solver,
                      "L": torch.empty((sp.H, sp.W), dtype=torch.uint8, device=self.device),
                      "R": torch.empty((sp.H, sp.W), dtype=torch.uint8, device=self.device)}
            self.state[stream] = st
        return st

    # --- request loop ----------------------------------------------------------------
    def submit(self, stream: int, left, right, t_arrival: Optional[float] = None) -> Request:
        with self.cv:
            req = Request(self._rid, stream, time.perf_counter() if t_arrival is None else t_arrival,
                          (left, right))
            self._rid += 1
            self.adm.push(req)
            self.cv.notify_all()
        return req

    def _dispatcher(self):
        with self.cv:
            while True:
                if self.closed and not self.adm.queue:
                    return
                nxt = self.adm.next() if self.free_slots else None
                if nxt is None:
                    self.cv.wait(timeout=0.05)
                    continue
                req, victims = nxt
                for s in victims:          # evicted state is dropped (memory returns to torch)
                    self.state.pop(s, None)
                slot = self.free_slots.pop(0)
                req.slot = slot
                req.t_admit = time.perf_counter()
                self._slot_req[slot] = req
                self.cv.notify_all()

    def _slot_loop(self, k: int):
        while True:
            with self.cv:
                while self._slot_req[k] is None:
                    if self.closed and not self.adm.queue and len(self.free_slots) == self.n_slots \
                            and self._stop:
                        return
                    self.cv.wait(timeout=0.05)
                req = self._slot_req[k]
            self._run(req)
            with self.cv:
                self._slot_req[k] = None
                self.adm.done(req)
                self.free_slots.append(req.slot)
                self.completed.append(req)
                self.cv.notify_all()

    def _run(self, req: Request):
        torch = self._torch
        cs = self.slot_streams[req.slot]
        try:
            with self.cv:
                st = self._ensure_state(req.stream, cs)
            left, right = req.payload
            with torch.cuda.stream(cs):
                st["L"].copy_(torch.as_tensor(left), non_blocking=True)
                st["R"].copy_(torch.as_tensor(right), non_blocking=True)
                res = st["solver"](st["L"], st["R"], stream=cs)
            cs.synchronize()
            req.t_done = time.perf_counter()
            if self.on_done is not None:
                self.on_done(req, res.D_f, res.C_f, res.mask)
        except Exception as e:  # reported, never swallowed silently
            req.status = -1
            req.t_done = time.perf_counter()
            self.errors.append(f"request {req.rid} (stream {req.stream}): {e}")

    def drain(self, timeout: float = 120.0):
        """Waits until every submitted request completed, then stops the dispatcher."""
        t_end = time.perf_counter() + timeout
        with self.cv:
            self.closed = True
            self.cv.notify_all()
            while (self.adm.queue or len(self.free_slots) < self.n_slots):
                if time.perf_counter() > t_end:
                    raise TimeoutError("requests still pending")
                self.cv.wait(timeout=0.05)
        self._dispatch.join(timeout=5.0)
        with self.cv:
            self._stop = True
            self.cv.notify_all()
        for t in self._threads:
            t.join(timeout=5.0)
        if self.errors:
            raise RuntimeError("; ".join(self.errors[:3]))


def replay(server: StereoServer, schedule, frames_for, time_scale: float = 1.0):
    """Submits (t_arrival, stream) events at their (scaled) wall-clock times. Returns the
    completed requests and the wall time of the run."""
    t0 = time.perf_counter()
    for (t, s) in schedule:
        target = t0 + t * time_scale
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        left, right = frames_for(s)
        server.submit(s, left, right, t_arrival=target)
    server.drain()
    return list(server.completed), time.perf_counter() - t0
