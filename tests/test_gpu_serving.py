"""GPU: the continuous-batching server (admission by memory budget, per-stream resident
state, eviction under a tight budget, frames of different sizes solved together by the
stage-batched solver, two lanes whose batches overlap on the device) returns for every
frame exactly what solving that frame alone returns, and what the oracle computes."""
import sys
import threading

import numpy as np
import pytest
import torch

import scenes
from oracle_cache import assert_equals_oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-serving]", *a, file=sys.stderr, flush=True)


def _streams():
    sizes = [(160, 120), (320, 240), (256, 192)]
    specs, frames = {}, {}
    from paper_1511_00758_amd.serving import StreamSpec
    for s in range(6):
        W, H = sizes[s % 3]
        prm = scenes.params_of(2, d_max=63 if W < 300 else 95)
        specs[s] = StreamSpec(W, H, prm)
        frames[s] = []
        for k in range(2):
            sc = scenes.make_rect_scene(W, H, seed=5000 + 10 * s + k, n_rects=6, dlo=2.0, dhi=60.0)
            frames[s].append((sc.left, sc.right))
    return specs, frames


@pytest.mark.parametrize("time_scale,per_stream", [(1.0, 1), (0.0, 2)])
def test_served_frames_equal_solo_solves_and_oracle(time_scale, per_stream):
    """Real-time arrivals (small batches, lanes overlapping) and all arrivals at once
    (large mixed-size batches, two frames of a stream in one batch)."""
    from paper_1511_00758_amd import api
    from paper_1511_00758_amd.serving import StereoServer, replay
    specs, frames = _streams()
    results = {}
    lock = threading.Lock()

    def on_done(req, D, C, M):
        with lock:
            results[req.rid] = (req.stream, req.payload, D.cpu().numpy(), C.cpu().numpy(), M.cpu().numpy(),
                                req.batch_size)

    # budget: room for about three streams' state, so streams are evicted and re-admitted
    probe = StereoServer(specs, budget_bytes=1 << 40, device=DEV)
    need = max(probe.state_bytes(s) for s in specs)
    probe.drain()
    server = StereoServer(specs, budget_bytes=3 * need * per_stream, device=DEV, on_done=on_done, n_lanes=2,
                          max_batch=8, frames_per_stream=per_stream)
    sched = scenes.stream_schedule(seed=7, n_streams=6, rate_hz=40.0, seconds=0.6)
    counter = {s: 0 for s in specs}

    def frames_for(s):
        f = frames[s][counter[s] % 2]
        counter[s] += 1
        return f

    done, wall = replay(server, sched, frames_for, time_scale=time_scale)
    sizes = [b for (_, b, _) in server.batches]
    _note(f"{len(done)} frames in {wall:.2f}s, {len(sizes)} batches (max {max(sizes)}), "
          f"lanes used {sorted({k for (k, _, _) in server.batches})}, evictions {server.adm.evictions}")
    assert len(done) == len(sched) and all(r.status == 0 for r in done)
    assert len(results) == len(sched)
    assert server.adm.evictions > 0
    if time_scale == 0.0:
        assert max(sizes) > 1                   # frames of several streams in one batch
        assert len({specs[r.stream].W for r in done if r.batch_size > 1}) > 1
        per_batch = {}
        for r in done:
            per_batch.setdefault(r.batch, []).append(r.stream)
        assert any(len(v) > len(set(v)) for v in per_batch.values())   # a stream twice in a batch
    for s in specs:                             # a stream's frames complete in arrival order
        mine = sorted((r for r in done if r.stream == s), key=lambda r: r.rid)
        assert all(a.t_done <= b.t_done for a, b in zip(mine, mine[1:]))
    solo, checked = {}, set()
    for rid, (s, (l, r), D, C, M, bsz) in sorted(results.items()):
        key = (s, counter_key(frames, s, l))
        if key not in solo:
            sp = specs[s]
            res = api.Solver(sp.W, sp.H, sp.params, device=DEV)(torch.from_numpy(l).to(DEV),
                                                               torch.from_numpy(r).to(DEV))
            torch.cuda.synchronize()
            solo[key] = (res.D_f.cpu().numpy(), res.C_f.cpu().numpy(), res.mask.cpu().numpy())
        sD, sC, sM = solo[key]
        assert (sD.view(np.uint32) == D.view(np.uint32)).all(), (rid, s, bsz)
        assert (sC == C).all(), (rid, s, bsz)
        assert (sM == M).all(), (rid, s, bsz)
        if key not in checked:                  # every distinct served frame against the oracle
            assert_equals_oracle(D, C, M, l, r, specs[s].params, f"(served frame {rid}, stream {s})")
            checked.add(key)
    assert len(checked) == 12


def counter_key(frames, s, l):
    """Which of the stream's two frames the payload is."""
    return 0 if frames[s][0][0] is l else 1
