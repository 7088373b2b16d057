"""GPU: sm_solve_many (one launch per stage over all frames) returns, for every frame of a
mixed batch, exactly what sm_solve returns for that frame alone, and what the oracle
computes."""
import sys

import numpy as np
import pytest
import torch

import scenes
from oracle_cache import assert_equals_oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-many]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _mixed():
    """Sizes 200x150 .. 1280x720, census windows 5x5 and 7x7, 1 and 3 iterations,
    disparity ranges 64..256, levels 1 and 3, a constant frame (no supports)."""
    out = []
    for f in range(2):
        sc = scenes.make_scene(1, scenes.seed_of(1, 30 + f))
        out.append((sc.left, sc.right, sc.params))
    for f in range(2):
        sc = scenes.make_scene(2, scenes.seed_of(2, 30 + f))
        out.append((sc.left, sc.right, dict(sc.params, levels=3 if f else 1)))
    sc = scenes.make_scene(3, scenes.seed_of(3, 30))
    out.append((sc.left, sc.right, sc.params))
    for k, (W, H, dr) in enumerate(((1280, 720, 256), (200, 150, 64), (333, 211, 192))):
        sc = scenes.make_rect_scene(W, H, seed=5000 + k, dlo=2.0, dhi=0.95 * dr)
        prm = scenes.params_of(4 if W > 300 else 2)
        prm.update(d_min=0, d_max=dr - 1)
        out.append((sc.left, sc.right, prm))
    flat = np.full((90, 120), 77, np.uint8)
    out.append((flat, flat.copy(), scenes.params_of(2)))
    return out


@pytest.fixture(scope="module")
def mixed():
    return _mixed()


def _solo(l, r, prm):
    from paper_1511_00758_amd import api
    H, W = l.shape
    res = api.Solver(W, H, prm, device=DEV)(_dev(l), _dev(r))
    torch.cuda.synchronize()
    return res.D_f.cpu().numpy(), res.C_f.cpu().numpy(), res.mask.cpu().numpy()


@pytest.mark.parametrize("threads", [1, 8])
def test_many_equals_solo(mixed, threads):
    from paper_1511_00758_amd import api
    _note("many threads", threads)
    ms = api.ManySolver(threads, device=DEV)
    outs, st = ms([(_dev(l), _dev(r), prm) for (l, r, prm) in mixed], stats=True, timing=True)
    torch.cuda.synchronize()
    total_valid = 0
    for i, ((l, r, prm), (D, C, M)) in enumerate(zip(mixed, outs)):
        sD, sC, sM = _solo(l, r, prm)
        assert (D.cpu().numpy().view(np.uint32) == sD.view(np.uint32)).all(), i
        assert (C.cpu().numpy() == sC).all(), i
        assert (M.cpu().numpy() == sM).all(), i
        total_valid += int(sM.sum())
    assert st["n_valid"] == total_valid
    # one launch per stage: two census windows, matching once, 3 iterations at most; the
    # batch is small enough for a star per wavefront (22.6k support candidates), so its star
    # kernels rasterise their own triangles and it has no raster stage
    assert st["stage_launches"]["census"] == 2 and st["stage_launches"]["match"] == 1
    assert st["stage_launches"]["validate"] == 3 and st["stage_launches"]["raster"] == 0


def test_many_against_oracle(mixed):
    """Frames of the mixed batch against the oracle, the 1280x720 pair with disparities
    0-255 (the largest size and range of the batched and serving workloads) included."""
    from paper_1511_00758_amd import api
    sub = [mixed[0], mixed[3], mixed[5], mixed[6]]
    assert sub[2][0].shape == (720, 1280) and sub[2][2]["d_max"] == 255
    outs = api.ManySolver(4, device=DEV)([(_dev(l), _dev(r), prm) for (l, r, prm) in sub])
    torch.cuda.synchronize()
    for (l, r, prm), (D, C, M) in zip(sub, outs):
        _note("many vs oracle", l.shape, prm["d_max"])
        assert_equals_oracle(D, C, M, l, r, prm, f"(sm_solve_many, {l.shape})")


def test_many_repeated_and_resized_batches(mixed):
    from paper_1511_00758_amd import api
    ms = api.ManySolver(4, device=DEV)
    frames = [(_dev(l), _dev(r), prm) for (l, r, prm) in mixed[:4]]
    first = [tuple(t.cpu().numpy() for t in o) for o in ms(frames)]
    for k in range(3):
        again = ms(frames if k != 1 else frames[:1])
        torch.cuda.synchronize()
        for a, b in zip(first, again):
            assert (a[0].view(np.uint32) == b[0].cpu().numpy().view(np.uint32)).all()
            assert (a[1] == b[1].cpu().numpy()).all() and (a[2] == b[2].cpu().numpy()).all()
    assert ms([]) == []


def test_many_rejects_fast_frames_before_work(mixed):
    from paper_1511_00758_amd import api, _lib
    l, r, prm = mixed[2]
    with pytest.raises((_lib.StereoMeshError, ValueError)):
        api.ManySolver(2, device=DEV)([(_dev(l), _dev(r), prm), (_dev(l), _dev(r), dict(prm, support_mode=1))])


def test_many_device_mesh_equals_host_mesh(mixed):
    """The tessellations of a batch built on the device (one workgroup per frame, one launch
    per iteration) give the same outputs as host triangulation, also with device and host
    frames mixed in one batch."""
    from paper_1511_00758_amd import api
    ms = api.ManySolver(8, device=DEV)
    runs = {}
    for mode in ("device", "host", "mixed"):
        _note("many mesh", mode)
        frames = []
        for i, (l, r, prm) in enumerate(mixed):
            hm = {"device": 0, "host": 1, "mixed": i % 2}[mode]
            frames.append((_dev(l), _dev(r), dict(prm, host_mesh=hm)))
        outs, st = ms(frames, stats=True, timing=True)
        torch.cuda.synchronize()
        runs[mode] = ([tuple(t.cpu().numpy() for t in o) for o in outs], st)
    dev_out, dev_st = runs["device"]
    for mode in ("host", "mixed"):
        out, st = runs[mode]
        assert st["n_tris"] == dev_st["n_tris"] and st["n_support"] == dev_st["n_support"]
        for a, b in zip(dev_out, out):
            assert (a[0].view(np.uint32) == b[0].view(np.uint32)).all()
            assert (a[1] == b[1]).all() and (a[2] == b[2]).all()
    # every frame built all its meshes on the device (the flat one: empty meshes), one launch
    # per tessellation round over the batch
    expect = sum(prm["n_iters"] for (l, r, prm) in mixed)
    assert dev_st["mesh_device"] == expect and dev_st["mesh_fallback"] == 0
    assert runs["host"][1]["mesh_device"] == 0
    assert dev_st["stage_launches"]["mesh"] == 3


def test_many_large_batch_grouped_stars_equal_solo():
    """A batch of 24 frames of the 640x480 workload: enough support candidates (about 74k)
    that the batched star kernel takes one star per 16-lane group; every frame bit-equal to
    its solo solve (one star per wavefront)."""
    from paper_1511_00758_amd import api
    scs = [scenes.make_scene(2, scenes.seed_of(2, 60 + f)) for f in range(4)]
    frames = [(_dev(scs[i % 4].left), _dev(scs[i % 4].right), scs[i % 4].params) for i in range(24)]
    solo = [_solo(sc.left, sc.right, sc.params) for sc in scs]
    _note("many grouped", len(frames))
    outs = api.ManySolver(8, device=DEV)(frames)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        got = tuple(t.cpu().numpy() for t in o)
        exp = solo[i % 4]
        assert (got[0].view(np.uint32) == exp[0].view(np.uint32)).all(), i
        assert (got[1] == exp[1]).all() and (got[2] == exp[2]).all(), i
