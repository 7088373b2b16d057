"""GPU: the serving loop (continuous admission over worker slots, per-stream resident
state, eviction under a tight budget) returns, for every frame, exactly what solving
that frame alone returns."""
import sys
import threading

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_served_frames_equal_solo_solves():
    from paper_1511_00758_amd import api
    from paper_1511_00758_amd.serving import StereoServer, StreamSpec, replay
    sizes = [(160, 120), (320, 240), (256, 192)]
    specs, frames = {}, {}
    for s in range(6):
        W, H = sizes[s % 3]
        prm = scenes.params_of(2, d_max=63 if W < 300 else 95)
        specs[s] = StreamSpec(W, H, prm)
        frames[s] = []
        for k in range(2):
            sc = scenes.make_rect_scene(W, H, seed=5000 + 10 * s + k, n_rects=6, dlo=2.0, dhi=60.0)
            frames[s].append((sc.left, sc.right))
    results = {}
    lock = threading.Lock()

    def on_done(req, D, C, M):
        with lock:
            results[req.rid] = (req.stream, req.payload, D.cpu().numpy(), C.cpu().numpy(), M.cpu().numpy())

    # budget: room for about three streams' state, so streams are evicted and re-admitted
    probe = StereoServer(specs, n_slots=1, budget_bytes=1 << 40, device=DEV)
    need = max(probe.state_bytes(s) for s in specs)
    probe.drain()
    server = StereoServer(specs, n_slots=3, budget_bytes=3 * need, device=DEV, on_done=on_done)
    sched = scenes.stream_schedule(seed=7, n_streams=6, rate_hz=40.0, seconds=0.6)
    counter = {s: 0 for s in specs}

    def frames_for(s):
        f = frames[s][counter[s] % 2]
        counter[s] += 1
        return f

    done, wall = replay(server, sched, frames_for)
    print(f"[gpu-serving] {len(done)} frames in {wall:.2f}s, evictions {server.adm.evictions}",
          file=sys.stderr, flush=True)
    assert len(done) == len(sched) and all(r.status == 0 for r in done)
    assert server.adm.evictions > 0
    solvers = {}
    for rid, (s, (l, r), D, C, M) in results.items():
        if s not in solvers:
            solvers[s] = api.Solver(specs[s].W, specs[s].H, specs[s].params, device=DEV)
        res = solvers[s](torch.from_numpy(l).to(DEV), torch.from_numpy(r).to(DEV))
        torch.cuda.synchronize()
        assert (res.D_f.cpu().numpy().view(np.uint32) == D.view(np.uint32)).all()
        assert (res.C_f.cpu().numpy() == C).all()
        assert (res.mask.cpu().numpy() == M).all()
