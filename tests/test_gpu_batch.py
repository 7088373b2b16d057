"""GPU: sm_solve_batch on mixed frames equals each frame solved alone (bit for bit), and
frames checked directly against the oracle."""
import sys

import numpy as np
import pytest
import torch

import scenes
from oracle_cache import assert_equals_oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-batch]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _mixed_frames():
    """Frames of uneven sizes and disparity ranges, as in the batched workload."""
    out = []
    for f in range(3):
        sc = scenes.make_scene(1, scenes.seed_of(1, 10 + f))
        out.append((sc.left, sc.right, sc.params))
    for f in range(2):
        sc = scenes.make_scene(2, scenes.seed_of(2, 10 + f))
        out.append((sc.left, sc.right, sc.params))
    sc = scenes.make_scene(3, scenes.seed_of(3, 10))
    out.append((sc.left, sc.right, sc.params))
    for k, (W, H, dr) in enumerate(((1280, 720, 256), (200, 150, 64), (333, 211, 192))):
        sc = scenes.make_rect_scene(W, H, seed=4000 + k, dlo=2.0, dhi=0.95 * dr)
        prm = scenes.params_of(4 if W > 300 else 2)
        prm.update(d_min=0, d_max=dr - 1)
        out.append((sc.left, sc.right, prm))
    return out


@pytest.fixture(scope="module")
def mixed():
    return _mixed_frames()


def _solo(l, r, prm):
    from paper_1511_00758_amd import api
    H, W = l.shape
    s = api.Solver(W, H, prm, device=DEV)
    res = s(_dev(l), _dev(r))
    torch.cuda.synchronize()
    return res.D_f.cpu().numpy(), res.C_f.cpu().numpy(), res.mask.cpu().numpy()


@pytest.mark.parametrize("workers", [1, 4, 9])
def test_batch_equals_solo(mixed, workers):
    from paper_1511_00758_amd import api
    _note("batch workers", workers)
    maxW = max(f[0].shape[1] for f in mixed)
    maxH = max(f[0].shape[0] for f in mixed)
    bs = api.BatchSolver(workers, maxW, maxH, [f[2] for f in mixed], device=DEV)
    frames = [(_dev(l), _dev(r), prm) for (l, r, prm) in mixed]
    outs, st, per = bs(frames, stats=True)
    torch.cuda.synchronize()
    assert {w for (w, _) in per} <= set(range(workers))
    for (l, r, prm), (D, C, M) in zip(mixed, outs):
        sD, sC, sM = _solo(l, r, prm)
        assert (D.cpu().numpy().view(np.uint32) == sD.view(np.uint32)).all()
        assert (C.cpu().numpy() == sC).all()
        assert (M.cpu().numpy() == sM).all()
    assert st["n_valid"] == sum(int(M.sum()) for (_, _, M) in outs)


def test_batch_against_oracle(mixed):
    """Frames of the concurrent batch against the oracle, the 1280x720 pair with
    disparities 0-255 included."""
    from paper_1511_00758_amd import api
    sub = [mixed[0], mixed[1], mixed[6], mixed[7]]
    assert sub[2][0].shape == (720, 1280) and sub[2][2]["d_max"] == 255
    bs = api.BatchSolver(3, 1280, 720, [f[2] for f in sub], device=DEV)
    outs = bs([(_dev(l), _dev(r), prm) for (l, r, prm) in sub])
    torch.cuda.synchronize()
    for (l, r, prm), (D, C, M) in zip(sub, outs):
        _note("batch vs oracle", l.shape, prm["d_max"])
        assert_equals_oracle(D, C, M, l, r, prm, f"(sm_solve_batch, {l.shape})")


def test_batch_rejects_bad_frames_before_work(mixed):
    from paper_1511_00758_amd import api, _lib
    l, r, prm = mixed[0]
    bs = api.BatchSolver(2, 320, 240, [prm], device=DEV)
    bad = dict(prm)
    bad["t_lo"] = prm["t_hi"] + 1
    with pytest.raises(_lib.StereoMeshError) as e:
        bs([(_dev(l), _dev(r), prm), (_dev(l), _dev(r), bad)])
    assert e.value.status == _lib.SM_ERR_ARG
    big = scenes.make_scene(2, scenes.seed_of(2, 20))
    with pytest.raises(_lib.StereoMeshError) as e:
        bs([(_dev(big.left), _dev(big.right), big.params)])
    assert e.value.status == _lib.SM_ERR_CAPACITY


def test_batch_repeated_calls_reuse_workers(mixed):
    from paper_1511_00758_amd import api
    sub = mixed[:3]
    bs = api.BatchSolver(3, 320, 240, [f[2] for f in sub], device=DEV)
    frames = [(_dev(l), _dev(r), prm) for (l, r, prm) in sub]
    first = [tuple(t.cpu().numpy() for t in o) for o in bs(frames)]
    for _ in range(5):
        again = bs(frames)
        torch.cuda.synchronize()
        for a, b in zip(first, again):
            assert all((x == y.cpu().numpy()).all() for x, y in zip(a, b) if x.dtype != np.float32)
            assert (a[0].view(np.uint32) == b[0].cpu().numpy().view(np.uint32)).all()
