"""Admission policy of the serving loop, driven by a simulated clock and a fake
device-memory budget (no GPU)."""
import heapq

import numpy as np
import pytest

from paper_1511_00758_amd.serving import Admission, Request


def _simulate(sizes, service, arrivals, budget, slots):
    """Event-driven run of the policy: returns completed requests and the peak of the
    resident bytes."""
    adm = Admission(budget, lambda s: sizes[s])
    events = [(t, 0, i) for i, (t, s) in enumerate(arrivals)]   # (time, kind 0=arrive 1=done, id)
    heapq.heapify(events)
    reqs = [Request(i, s, t) for i, (t, s) in enumerate(arrivals)]
    free = slots
    done, peak, order = [], 0, []
    while events:
        t, kind, i = heapq.heappop(events)
        if kind == 0:
            adm.push(reqs[i])
        else:
            adm.done(reqs[i])
            reqs[i].t_done = t
            done.append(reqs[i])
            free += 1
        while free > 0:
            nxt = adm.next()
            if nxt is None:
                break
            r, victims = nxt
            r.t_admit = t
            order.append((r.stream, r.rid, tuple(victims)))
            free -= 1
            peak = max(peak, adm.used)
            heapq.heappush(events, (t + service[r.stream], 1, r.rid))
    return done, peak, order, adm


def test_all_frames_complete_within_budget_and_in_stream_order():
    rng = np.random.default_rng(0)
    sizes = {s: [100, 250, 600][s % 3] for s in range(16)}
    service = {s: [1.0, 2.5, 6.0][s % 3] for s in range(16)}
    arrivals = sorted((float(t), s) for s in range(16) for t in np.cumsum(rng.exponential(33.0, 20)))
    done, peak, order, adm = _simulate(sizes, service, arrivals, budget=2000, slots=8)
    assert len(done) == len(arrivals)
    assert peak <= 2000
    for s in range(16):
        rids = [r.rid for r in sorted(done, key=lambda r: r.t_admit) if r.stream == s]
        assert rids == sorted(rids)                    # a stream's frames stay in order
    assert adm.evictions > 0                           # the budget forced evictions
    assert all(r.t_admit >= r.t_arrival and r.t_done > r.t_admit for r in done)


def test_one_frame_in_flight_per_stream():
    sizes = {0: 10, 1: 10}
    service = {0: 5.0, 1: 5.0}
    arrivals = [(0.0, 0), (0.1, 0), (0.2, 0), (0.3, 1)]
    done, _, order, _ = _simulate(sizes, service, arrivals, budget=100, slots=4)
    admits = {r.rid: r.t_admit for r in done}
    assert admits[1] >= 5.0 and admits[2] >= 10.0    # stream 0 serialised
    assert admits[3] == pytest.approx(0.3)           # stream 1 overlaps


def test_lru_eviction_and_no_head_of_line_blocking():
    adm = Admission(100, lambda s: {0: 40, 1: 40, 2: 60, 3: 30}[s])
    for rid, s in enumerate([0, 1]):
        adm.push(Request(rid, s, 0.0))
    r0, _ = adm.next()
    r1, _ = adm.next()
    adm.done(r0)
    adm.done(r1)                                   # both resident (80 used), idle; 0 is LRU
    adm.push(Request(2, 2, 1.0))                   # needs 60: must evict
    r2, victims = adm.next()
    assert r2.rid == 2 and victims == [0]          # least recently used goes first
    assert adm.used == 100
    adm.push(Request(3, 3, 2.0))                   # needs 30: stream 2 is busy, stream 1 idle
    adm.push(Request(4, 1, 2.1))                   # stream 1 is resident at this point
    nxt = adm.next()
    assert nxt is not None
    r, victims = nxt
    # stream 3 (30 B) fits after evicting idle stream 1 (40 B): admitted first, FIFO
    assert r.rid == 3 and victims == [1]
    adm.done(r2)
    r4, victims4 = adm.next()
    assert r4.rid == 4 and victims4 == [2]


def test_resident_stream_not_blocked_by_memory_wait():
    adm = Admission(100, lambda s: {0: 60, 1: 60, 2: 30}[s])
    adm.push(Request(0, 0, 0.0))
    r0, _ = adm.next()                             # stream 0 busy, 60 used
    adm.push(Request(1, 2, 0.1))
    r1, _ = adm.next()                             # stream 2 fits (90 used)
    adm.done(r1)                                   # stream 2 idle, resident
    adm.push(Request(2, 1, 0.2))                   # stream 1 (60) cannot fit while 0 is busy
    adm.push(Request(3, 2, 0.3))                   # stream 2 is resident: may go ahead
    r, victims = adm.next()
    assert r.rid == 3 and victims == []
    assert adm.next() is None                      # request 2 still waits for memory


def test_oversized_stream_rejected():
    adm = Admission(50, lambda s: 80)
    with pytest.raises(ValueError):
        adm.push(Request(0, 0, 0.0))


def test_next_batch_takes_every_admissible_frame_once_per_stream():
    """A free lane takes every admissible waiting frame: the oldest frame of each stream
    that is not busy and fits the budget (after evicting idle streams), up to the batch
    limit, in arrival order; later frames of a stream wait for its current one."""
    sizes = {0: 10, 1: 10, 2: 10, 3: 25}
    adm = Admission(40, lambda s: sizes[s])
    reqs = [Request(i, s, float(i)) for i, s in enumerate([0, 0, 1, 2, 3, 1])]
    for r in reqs:
        adm.push(r)
    batch, evicted = adm.next_batch(8)
    assert [r.rid for r in batch] == [0, 2, 3]      # stream 3 does not fit beside three busy ones
    assert evicted == [] and adm.used == 30
    assert adm.next_batch(8) == ([], [])            # streams 0, 1, 2 are busy, 3 still waits
    for r in batch:
        adm.done(r)
    batch2, _ = adm.next_batch(1)                   # the limit: the oldest admissible frame
    assert [r.rid for r in batch2] == [1]
    batch3, evicted3 = adm.next_batch(8)            # stream 3 evicts idle 1 and 2; then 1 cannot return
    assert [r.rid for r in batch3] == [4] and evicted3 == [1, 2]
    assert adm.used == 35
    for r in batch2 + batch3:
        adm.done(r)
    batch4, evicted4 = adm.next_batch(8)
    assert [r.rid for r in batch4] == [5] and evicted4 == [0]


def test_next_batch_evicts_idle_streams_lru():
    sizes = {s: 10 for s in range(5)}
    adm = Admission(30, lambda s: sizes[s])
    for i, s in enumerate([0, 1, 2]):
        adm.push(Request(i, s, float(i)))
    first, _ = adm.next_batch(8)
    for r in first:
        adm.done(r)
    adm.push(Request(3, 3, 3.0))
    adm.push(Request(4, 4, 4.0))
    adm.push(Request(5, 0, 5.0))
    batch, evicted = adm.next_batch(8)
    assert [r.rid for r in batch] == [3, 4, 5]
    assert evicted == [0, 1, 2] and adm.evictions == 3   # 3 evicts 0, 4 evicts 1, 0 returns evicting 2
    assert adm.used <= 30


def test_next_batch_several_frames_of_a_stream_in_order():
    """With per_stream = k, a backlogged stream contributes its k oldest frames to one
    batch (in arrival order); its later frames wait until that batch is done."""
    adm = Admission(100, lambda s: 10)
    order = [0, 0, 1, 0, 0, 1, 1, 1, 0]
    reqs = [Request(i, s, float(i)) for i, s in enumerate(order)]
    for r in reqs:
        adm.push(r)
    batch, _ = adm.next_batch(16, per_stream=3)
    assert [r.rid for r in batch] == [0, 1, 2, 3, 5, 6]
    assert adm.next_batch(16, per_stream=3) == ([], [])
    for r in batch:
        adm.done(r)
    batch2, _ = adm.next_batch(16, per_stream=3)
    assert [r.rid for r in batch2] == [4, 7, 8]
