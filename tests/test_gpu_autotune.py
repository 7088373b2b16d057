"""GPU: the autotuner (sm_autotune) picks launch shapes among its candidates for a frame
size, and solves after tuning give bit for bit what solves before it gave (a launch shape
changes speed only), for the tuned frame and for another frame of the same size."""
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_autotune_keeps_outputs():
    from paper_1511_00758_amd import api
    frames = [scenes.make_scene(2, scenes.seed_of(2, 40 + k)) for k in range(2)]
    H, W = frames[0].left.shape
    prm = frames[0].params
    before = []
    for sc in frames:
        r = api.Solver(W, H, prm, device=DEV)(_dev(sc.left), _dev(sc.right))
        torch.cuda.synchronize()
        before.append(tuple(t.cpu().numpy().copy() for t in (r.D_f, r.C_f, r.mask)))
    solver = api.Solver(W, H, prm, device=DEV)
    print("[gpu-autotune] tuning", W, H, file=sys.stderr, flush=True)
    ch = solver.autotune(_dev(frames[0].left), _dev(frames[0].right))
    torch.cuda.synchronize()
    assert len(ch["validate_waves"]) == prm["n_iters"]
    assert all(w in (1, 2, 4, 8, 16) for w in ch["validate_waves"])
    assert ch["raster_blocks"] in (512, 1024, 2048, 4096, 8192)
    # the tuning call leaves the frame's results in the outputs
    tuned0 = tuple(t.cpu().numpy() for t in (solver.D_f, solver.C_f, solver.mask))
    for k, sc in enumerate(frames):
        r = solver(_dev(sc.left), _dev(sc.right))
        torch.cuda.synchronize()
        got = tuple(t.cpu().numpy() for t in (r.D_f, r.C_f, r.mask))
        assert (got[0].view(np.uint32) == before[k][0].view(np.uint32)).all(), k
        assert (got[1] == before[k][1]).all() and (got[2] == before[k][2]).all(), k
    assert (tuned0[0].view(np.uint32) == before[0][0].view(np.uint32)).all()
    assert (tuned0[1] == before[0][1]).all() and (tuned0[2] == before[0][2]).all()
