"""Continuous-batching request loop for many simulated camera streams.

Frames arrive per camera stream. Whenever one of ``n_lanes`` execution lanes is free,
every admissible waiting frame (up to ``max_batch``) is taken at once and solved as one
stage-batched batch (``sm_solve_many``: one kernel launch per stage over all frames of
the batch, frames of different sizes together). Frames that arrive while batches are on
the GPU wait for the next free lane, so work keeps flowing in as the device frees up;
with two or more lanes, batches overlap on the device (each lane has its own host
thread, HIP stream and batch workspace, and the library releases the GIL while it
runs).

Each stream keeps its state resident on the device between frames (``frames_per_stream``
slots of an input pair and output maps, and their share of the batch workspaces in the
budget); a stream is admitted only when that state fits the HBM budget, after evicting
idle streams least recently used. A stream's frames are solved in arrival order: up to
``frames_per_stream`` of its oldest waiting frames go into one batch (and complete
together), and its next frames wait until that batch is done.

``Admission`` is the host-side policy alone (no GPU): it is driven by the server, and by
the CPU tests with a simulated clock and a fake budget. ``StereoServer`` executes
admitted batches with the library; every step of the method runs in the library.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Tuple


@dataclass
class Request:
    rid: int
    stream: int
    t_arrival: float
    payload: object = None          # (left, right) host arrays or tensors
    t_admit: float = 0.0
    t_done: float = 0.0
    lane: int = -1
    batch: int = -1                 # id of the batch that solved it
    batch_size: int = 0
    status: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Admission:
    """FIFO admission under a device-memory budget with resident per-stream state.

    ``state_bytes(stream)`` gives the bytes a stream needs while resident. A request is
    admissible when its stream is not busy and either its state is resident or can be
    made resident (budget permitting) after evicting idle resident streams in
    least-recently-used order. Requests are considered in arrival order; a request that
    cannot be admitted does not block later requests of other streams whose state is
    already resident (no head-of-line blocking on memory)."""

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
        batch, evicted = self.next_batch(1)
        return (batch[0], evicted) if batch else None

    def _admit(self, stream: int) -> Optional[List[int]]:
        """Makes ``stream`` resident (evicting idle streams if needed); returns the evicted
        streams, or None when its state does not fit beside the busy ones."""
        if stream in self.resident:
            victims = []
        else:
            victims = self._make_room(self.state_bytes(stream))
            if victims is None:
                return None
        for s in victims:
            self.used -= self.resident.pop(s)
            self.evictions += 1
        if stream not in self.resident:
            b = self.state_bytes(stream)
            self.resident[stream] = b
            self.used += b
        self.resident.move_to_end(stream)
        return victims

    def next_batch(self, max_frames: int, per_stream: int = 1) -> Tuple[List[Request], List[int]]:
        """Pops up to ``max_frames`` admissible requests in arrival order: of each stream
        that is not busy, its oldest waiting frames, at most ``per_stream`` of them (a
        stream's frames then complete together, in order); returns them with every stream
        evicted to make room. Their streams are busy until ``done``."""
        batch, evicted, taken, blocked = [], [], {}, set()
        i = 0
        while i < len(self.queue) and len(batch) < max_frames:
            r = self.queue[i]
            s = r.stream
            if s in taken:
                ok = taken[s] < per_stream and s not in blocked
            else:
                ok = s not in self.busy and s not in blocked
                if ok:
                    victims = self._admit(s)    # streams taken so far are busy: never evicted
                    if victims is None:
                        ok = False
                    else:
                        evicted += victims
                        self.busy.add(s)
                        taken[s] = 0
            if not ok:
                blocked.add(s)                  # its later frames wait behind this one
                i += 1
                continue
            taken[s] += 1
            batch.append(r)
            del self.queue[i]
        return batch, evicted

    def done(self, req: Request):
        self.busy.discard(req.stream)


@dataclass
class StreamSpec:
    W: int
    H: int
    params: dict


class StereoServer:
    """Serves camera streams by continuous batching over ``n_lanes`` execution lanes.

    ``specs[stream]`` gives each camera stream's frame size and method parameters (grid
    supports; every tessellation on the device). ``on_done(req, D_f, C_f, mask)`` is
    called on the lane's thread once the frame's outputs are complete (device tensors of
    the stream's resident state, valid until that stream's next frame)."""

    def __init__(self, specs: Dict[int, StreamSpec], budget_bytes: int, device="cuda:0", on_done=None,
                 n_lanes: int = 2, max_batch: int = 32, frames_per_stream: int = 1, host_threads: int = 4):
        import torch
        from . import api
        self._torch = torch
        self._api = api
        self.specs = {s: StreamSpec(sp.W, sp.H, dict(sp.params, host_mesh=0, support_mode=0))
                      for s, sp in specs.items()}
        self.device = device
        self.on_done = on_done
        self.max_batch = int(max_batch)
        self.per_stream = int(frames_per_stream)
        lib = api._lib.load()
        self._ws_need = {s: int(lib.sm_solve_workspace_bytes(sp.W, sp.H, api.make_params(sp.params)))
                         for s, sp in self.specs.items()}
        if any(v == 0 for v in self._ws_need.values()):
            raise ValueError("invalid stream size or parameters")
        self.adm = Admission(budget_bytes, self.state_bytes)
        self.n_lanes = int(n_lanes)
        self.cv = threading.Condition()
        self.state: Dict[int, dict] = {}
        self.completed: List[Request] = []
        self.batches: List[Tuple[int, int, float]] = []   # (lane, frames, device seconds)
        self.closed = False
        self._stop = False
        self.errors: List[str] = []
        self._rid = 0
        self._n_batches = 0
        self._lane_batch: List[Optional[List[Request]]] = [None] * self.n_lanes
        self._lanes = [{"stream": torch.cuda.Stream(device=device),
                        "solver": api.ManySolver(host_threads, device=device)} for _ in range(self.n_lanes)]
        self._threads = [threading.Thread(target=self._lane_loop, args=(k,), daemon=True)
                         for k in range(self.n_lanes)]
        for t in self._threads:
            t.start()
        self._dispatch = threading.Thread(target=self._dispatcher, daemon=True)
        self._dispatch.start()

    # --- memory accounting -----------------------------------------------------------
    def state_bytes(self, stream: int) -> int:
        """Per frame slot of the stream: inputs (2 B/px) and outputs (6 B/px) kept
        resident, plus the frame's share of a batch workspace (what sm_solve would need
        for it alone); ``frames_per_stream`` slots."""
        sp = self.specs[stream]
        return self.per_stream * (self._ws_need[stream] + sp.W * sp.H * (2 + 4 + 1 + 1))

    def _ensure_state(self, stream: int):
        st = self.state.get(stream)
        if st is None:
            torch = self._torch
            sp = self.specs[stream]
            dev = self.device
            st = [{"L": torch.empty((sp.H, sp.W), dtype=torch.uint8, device=dev),
                   "R": torch.empty((sp.H, sp.W), dtype=torch.uint8, device=dev),
                   "out": (torch.empty((sp.H, sp.W), dtype=torch.float32, device=dev),
                           torch.empty((sp.H, sp.W), dtype=torch.uint8, device=dev),
                           torch.empty((sp.H, sp.W), dtype=torch.uint8, device=dev))}
                  for _ in range(self.per_stream)]
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
        torch = self._torch
        with self.cv:
            while True:
                if self.closed and not self.adm.queue:
                    return
                free = [k for k in range(self.n_lanes) if self._lane_batch[k] is None]
                batch, evicted = self.adm.next_batch(self.max_batch, self.per_stream) if free else ([], [])
                if not batch:
                    self.cv.wait(timeout=0.02)
                    continue
                for s in evicted:            # evicted state is dropped (memory returns to torch)
                    self.state.pop(s, None)
                fresh = [r.stream for r in batch if r.stream not in self.state]
                for s in fresh:
                    self._ensure_state(s)
                if fresh:                    # new buffers are ready before any lane stream uses them
                    torch.cuda.current_stream(self.device).synchronize()
                now = time.perf_counter()
                k = free[0]
                for r in batch:
                    r.t_admit = now
                    r.lane = k
                    r.batch = self._n_batches
                    r.batch_size = len(batch)
                self._n_batches += 1
                self._lane_batch[k] = batch
                self.cv.notify_all()

    def _lane_loop(self, k: int):
        while True:
            with self.cv:
                while self._lane_batch[k] is None:
                    if self._stop:
                        return
                    self.cv.wait(timeout=0.02)
                batch = self._lane_batch[k]
                states, slot = [], {}
                for r in batch:                 # a stream's frames take its slots in order
                    j = slot.get(r.stream, 0)
                    slot[r.stream] = j + 1
                    states.append(self.state[r.stream][j])
            self._run(k, batch, states)
            with self.cv:
                for r in batch:
                    self.adm.done(r)
                    self.completed.append(r)
                self._lane_batch[k] = None
                self.cv.notify_all()

    def _run(self, k: int, batch: List[Request], states: List[dict]):
        torch = self._torch
        lane = self._lanes[k]
        cs = lane["stream"]
        try:
            t0 = time.perf_counter()
            frames, outs = [], []
            with torch.cuda.stream(cs):
                for r, st in zip(batch, states):
                    left, right = r.payload
                    st["L"].copy_(torch.as_tensor(left), non_blocking=True)
                    st["R"].copy_(torch.as_tensor(right), non_blocking=True)
                    frames.append((st["L"], st["R"], self.specs[r.stream].params))
                    outs.append(st["out"])
                lane["solver"](frames, outputs=outs, stream=cs)   # synchronises cs at its end
            t1 = time.perf_counter()
            for r in batch:
                r.t_done = t1
            self.batches.append((k, len(batch), t1 - t0))
            if self.on_done is not None:
                for r, st in zip(batch, states):
                    self.on_done(r, *st["out"])
        except Exception as e:  # reported, never swallowed silently
            t1 = time.perf_counter()
            for r in batch:
                r.status = -1
                r.t_done = t1
            self.errors.append(f"batch of {len(batch)} on lane {k}: {e}")

    def drain(self, timeout: float = 120.0):
        """Waits until every submitted request completed, then stops the loop's threads."""
        t_end = time.perf_counter() + timeout
        with self.cv:
            self.closed = True
            self.cv.notify_all()
            while self.adm.queue or any(b is not None for b in self._lane_batch):
                if time.perf_counter() > t_end:
                    raise TimeoutError("requests still pending")
                self.cv.wait(timeout=0.02)
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
