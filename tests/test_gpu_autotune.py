"""GPU: the autotuner (sm_autotune) picks launch shapes among its candidates for a frame
size, and solves after tuning give bit for bit what solves before it gave (a launch shape
changes speed only), for the tuned frame and for another frame of the same size; every
matcher and census shape, forced, gives the default results."""
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
    assert ch["raster_blocks"] == 0  # (no solve launches the bounded-grid rasteriser)
    assert ch["match_lanes"] in (16, 32, 64) and ch["census_rows"] in (8, 16, 32)
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


def _outputs(res):
    return tuple(t.cpu().numpy().copy() for t in res)


def test_every_match_and_census_shape_gives_the_same_results():
    """The matcher's lanes per candidate (64, 32, 16) and the census tile rows (8, 16, 32),
    forced with sm_set_launch_shape, give bit for bit the default results: a 640x480 frame
    (disparities 0-127) by sm_solve, and a batch of four frames of three sizes and
    disparity ranges 0-63 / 0-127 / 0-255 by sm_solve_many."""
    from paper_1511_00758_amd import api
    sc = scenes.make_scene(2, scenes.seed_of(2, 50))
    H, W = sc.left.shape
    prm = sc.params
    l, r = _dev(sc.left), _dev(sc.right)
    solver = api.Solver(W, H, prm, device=DEV)
    base = _outputs((lambda x: (x.D_f, x.C_f, x.mask))(solver(l, r)))
    batch = []
    for k, ((bw, bh), dmax) in enumerate((((320, 240), 63), ((640, 480), 127), ((1242, 375), 255),
                                          ((320, 240), 255))):
        s2 = scenes.make_rect_scene(bw, bh, seed=900 + k, dlo=2.0, dhi=0.9 * (dmax + 1))
        batch.append((_dev(s2.left), _dev(s2.right), scenes.params_of(4, d_min=0, d_max=dmax)))
    ms = api.ManySolver(4, device=DEV)
    base_many = [_outputs(o) for o in ms(batch)]
    torch.cuda.synchronize()
    sizes = {(W, H)} | {(b[0].shape[1], b[0].shape[0]) for b in batch}

    def set_all(lanes, rows):
        for (bw, bh) in sizes:
            for dmax in (63, 127, 255):
                api.set_launch_shape("match_lanes", bw, bh, dmax + 1, lanes)
            api.set_launch_shape("census_rows", bw, bh, 3 << 8 | 3, rows)

    try:
        for lanes, rows in ((16, 8), (32, 32), (64, 16), (16, 32)):
            print("[gpu-autotune] shapes", lanes, rows, file=sys.stderr, flush=True)
            set_all(lanes, rows)
            got = _outputs((lambda x: (x.D_f, x.C_f, x.mask))(solver(l, r)))
            assert (got[0].view(np.uint32) == base[0].view(np.uint32)).all(), (lanes, rows)
            assert (got[1] == base[1]).all() and (got[2] == base[2]).all(), (lanes, rows)
            for k, o in enumerate(ms(batch)):
                g = _outputs(o)
                assert (g[0].view(np.uint32) == base_many[k][0].view(np.uint32)).all(), (lanes, rows, k)
                assert (g[1] == base_many[k][1]).all() and (g[2] == base_many[k][2]).all(), (lanes, rows, k)
    finally:
        set_all(0, 0)
