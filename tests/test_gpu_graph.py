"""GPU: a stage-batched solve captured into a HIP graph (sm_solve_many_capture) and replayed
(sm_many_graph_run). Every replay -- with new image contents copied into the captured input
buffers, and eager work and synchronisations between the replays -- gives for every frame
exactly what sm_solve gives for that frame alone, and one frame of every replay equals
the oracle."""
import sys

import numpy as np
import pytest
import torch

import scenes
from oracle_cache import assert_equals_oracle
from test_gpu_many import _mixed, _solo

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-graph]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# image contents of the successive runs: rows are independent epipolar lines, so flipping
# both images upside down or shifting both by whole columns gives valid pairs of the same size
_VIEWS = [lambda a: a, np.flipud, lambda a: np.roll(a, 7, axis=1), lambda a: a]
# the frame of each run that is also compared with the oracle
_ORACLE_FRAME = [5, 0, 3, 7]


def test_graph_replays_equal_solo():
    from paper_1511_00758_amd import api
    mixed = _mixed()
    Ls = [_dev(l) for (l, _, _) in mixed]
    Rs = [_dev(r) for (_, r, _) in mixed]
    ms = api.ManySolver(device=DEV)
    _note("capture", len(mixed), "frames")
    outs, graph = ms.capture([(L, R, prm) for L, R, (_, _, prm) in zip(Ls, Rs, mixed)])
    torch.cuda.synchronize()
    try:
        for k, view in enumerate(_VIEWS):
            if k > 0:
                for L, R, (l, r, _) in zip(Ls, Rs, mixed):
                    L.copy_(_dev(view(l)))
                    R.copy_(_dev(view(r)))
                # eager work of the program between replays
                l0, r0, p0 = mixed[0]
                api.Solver(l0.shape[1], l0.shape[0], p0, device=DEV)(_dev(r0), _dev(l0))
                torch.cuda.synchronize()
                _note("replay", k)
                st = graph.run(stats=True)
                torch.cuda.synchronize()
            else:
                st = None
            # one frame of every run against the oracle (the 1280x720, d 0-255 pair first)
            i_or = _ORACLE_FRAME[k]
            l, r, prm = mixed[i_or]
            _note("replay", k, "frame", i_or, l.shape, "vs oracle")
            assert_equals_oracle(*outs[i_or], view(l), view(r), prm, f"(graph run {k}, frame {i_or})")
            total = 0
            for i, ((l, r, prm), (D, C, M)) in enumerate(zip(mixed, outs)):
                sD, sC, sM = _solo(view(l), view(r), prm)
                assert (D.cpu().numpy().view(np.uint32) == sD.view(np.uint32)).all(), (k, i)
                assert (C.cpu().numpy() == sC).all(), (k, i)
                assert (M.cpu().numpy() == sM).all(), (k, i)
                total += int(sM.sum())
            if st is not None:
                assert st["n_valid"] == total
                assert st["mesh_fallback"] == 0
    finally:
        graph.close()


def test_graph_capture_needs_device_meshes():
    from paper_1511_00758_amd import api, _lib
    mixed = _mixed()[:2]
    frames = [(_dev(l), _dev(r), dict(prm, host_mesh=i)) for i, (l, r, prm) in enumerate(mixed)]
    with pytest.raises(_lib.StereoMeshError):
        api.ManySolver(device=DEV).capture(frames)


def test_graph_256_frames_sampled():
    """A batch of 256 frames of the 640x480 workload (8 scenes cycled), as many mesh
    workgroups as the chip has CUs; two replays, sampled frames and the valid-pixel total
    against the per-frame solver."""
    from paper_1511_00758_amd import api
    scs = [scenes.make_scene(2, scenes.seed_of(2, f)) for f in range(8)]
    pairs = [(_dev(sc.left), _dev(sc.right)) for sc in scs]
    frames = [(pairs[i % 8][0], pairs[i % 8][1], scs[i % 8].params) for i in range(256)]
    solo = [_solo(sc.left, sc.right, sc.params) for sc in scs]
    _note("capture 256 frames")
    outs, graph = api.ManySolver(device=DEV).capture(frames)
    try:
        for rep in range(2):
            st = graph.run(stats=True)
            torch.cuda.synchronize()
            assert st["mesh_fallback"] == 0
            assert st["n_valid"] == 32 * sum(int(m.sum()) for (_, _, m) in solo)
            for i in (0, 9, 130, 255):
                D, C, M = outs[i]
                sD, sC, sM = solo[i % 8]
                assert (D.cpu().numpy().view(np.uint32) == sD.view(np.uint32)).all(), (rep, i)
                assert (C.cpu().numpy() == sC).all(), (rep, i)
                assert (M.cpu().numpy() == sM).all(), (rep, i)
    finally:
        graph.close()
