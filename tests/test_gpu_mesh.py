"""Device meshes (Sec. III-A / Alg. 1: the first mesh built on the device from the grid
supports, the later tessellations inserted into it) against the host triangulation: the
perturbed Delaunay triangulation is unique, so a solve whose tessellations run on the
device must give the same triangle counts and bit-identical outputs as one that
triangulates every iteration on the host; the solve parity tests compare the device path
with the oracle as well."""
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-mesh]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _solve(sc, prm):
    from paper_1511_00758_amd import api
    H, W = sc.left.shape
    r = api.Solver(W, H, prm, device=DEV)(_dev(sc.left), _dev(sc.right), stats=True)
    torch.cuda.synchronize()
    return r.D_f.cpu().numpy(), r.C_f.cpu().numpy(), r.mask.cpu().numpy(), r.stats


def _check(sc, prm):
    dev = _solve(sc, dict(prm, host_mesh=0))
    host = _solve(sc, dict(prm, host_mesh=1))
    n_iters = prm["n_iters"]
    assert dev[3]["n_support"] == host[3]["n_support"]
    assert dev[3]["n_tris"] == host[3]["n_tris"]
    for a, b in zip(dev[:3], host[:3]):
        assert (a.view(np.uint8) == b.view(np.uint8)).all()
    assert host[3]["mesh_device"] == 0
    assert dev[3]["mesh_fallback"] == 0
    assert dev[3]["mesh_device"] == n_iters  # every tessellation on the device (grid or FAST supports)
    return dev[3]


@pytest.mark.parametrize("cfg,frame", [(2, 0), (2, 1), (2, 2), (3, 0), (3, 2)])
def test_device_mesh_equals_host(cfg, frame):
    _note("scene", cfg, frame)
    sc = scenes.make_scene(cfg, scenes.seed_of(cfg, frame))
    _check(sc, sc.params)


@pytest.mark.parametrize("n_iters,sz0", [(5, 32), (7, 16), (8, 8)])
def test_device_mesh_deep_iterations(n_iters, sz0):
    """Many iterations down to 1 px cells: dense batches of new supports, many of them in
    the same triangle and on shared edges."""
    _note("deep", n_iters, sz0)
    sc = scenes.make_rect_scene(200, 150, seed=n_iters * 31 + sz0, n_rects=8, dlo=2.0, dhi=40.0)
    prm = dict(scenes.params_of(2), n_iters=n_iters, sz_occ0=sz0, d_max=63, t_hi=10, t_lo=8)
    st = _check(sc, prm)
    assert st["n_support"][-1] > st["n_support"][0]


def test_device_mesh_loose_thresholds():
    """t_lo = t_hi: every validated cell with a good pixel adds a support, so the later
    batches are large and tie-heavy (supports on a regular lattice of cells)."""
    _note("loose")
    sc = scenes.make_scene(2, scenes.seed_of(2, 4), t_hi=24, t_lo=24)
    _check(sc, sc.params)


def test_device_mesh_fast_supports():
    """Irregular first mesh: FAST keypoints from spatial bins instead of the grid."""
    _note("fast")
    sc = scenes.make_scene(2, scenes.seed_of(2, 5))
    _check(sc, dict(sc.params, support_mode=1, fast_threshold=12))


@pytest.mark.parametrize("W,H", [(1280, 720), (1920, 1080)])
def test_device_mesh_serving_sizes(W, H):
    """The serving workload's larger frames (d 0-255, 3 iterations): tens of thousands of
    supports in the last tessellation."""
    _note("serving", W, H)
    sc = scenes.make_rect_scene(W, H, seed=W + 7, dlo=2.0, dhi=240.0)
    st = _check(sc, scenes.params_of(5))
    assert st["n_support"][-1] > 10000 or W < 1920


@pytest.mark.parametrize("W,H", [(320, 4200), (2560, 1440)])
def test_device_mesh_counts_outside_lds(W, H):
    """Frames whose rows (more than 4096) or bucket cells (more than 12288) do not fit the
    preparation kernel's LDS: its counts and row extremes go to global memory."""
    _note("prep in global memory", W, H)
    sc = scenes.make_rect_scene(W, H, seed=W + H, dlo=2.0, dhi=120.0)
    _check(sc, scenes.params_of(3) if W > 640 else scenes.params_of(2))


def test_device_mesh_repeated_solves_reuse_workspace():
    """One solver, frames of different content in a row: nothing of the previous frame's
    mesh survives in the workspace."""
    from paper_1511_00758_amd import api
    _note("reuse")
    frames = [scenes.make_scene(2, scenes.seed_of(2, f)) for f in (6, 7, 6)]
    H, W = frames[0].left.shape
    solver = api.Solver(W, H, frames[0].params, device=DEV)
    outs = []
    for sc in frames:
        r = solver(_dev(sc.left), _dev(sc.right), stats=True)
        torch.cuda.synchronize()
        outs.append((r.D_f.cpu().numpy().copy(), r.stats["n_tris"]))
    ref = _solve(frames[0], dict(frames[0].params, host_mesh=1))
    assert outs[0][1] == ref[3]["n_tris"] == outs[2][1]
    assert (outs[0][0].view(np.uint32) == ref[0].view(np.uint32)).all()
    assert (outs[2][0].view(np.uint32) == outs[0][0].view(np.uint32)).all()


def test_device_mesh_fan_hub_against_oracle():
    """One mesh vertex owning 122 triangles of the first tessellation (a fan from a single
    point over a row of points): the star kernel writes them in full sets and rasterises
    those sets after its walk; D_f, C_f and mask equal the oracle's bit for bit."""
    import oracle
    from paper_1511_00758_amd import api
    left, right = scenes.fan_pair(1280, 480, seed=77)
    prm = scenes.params_of(2)
    _note("fan hub 1280x480")
    r = api.Solver(1280, 480, prm, device=DEV)(_dev(left), _dev(right), stats=True)
    torch.cuda.synchronize()
    assert r.stats["n_tris"][0] == 122 and r.stats["mesh_device"] == prm["n_iters"]
    assert r.stats["mesh_fallback"] == 0
    ref = oracle.solve(left, right, oracle.Params.from_dict(prm))
    assert (r.D_f.cpu().numpy().view(np.uint32) == ref["D_f"].view(np.uint32)).all()
    assert (r.C_f.cpu().numpy() == ref["C_f"]).all()
    assert (r.mask.cpu().numpy().astype(bool) == ref["mask"]).all()


@pytest.mark.parametrize("W,n", [(1280, 12), (3200, 5)])
def test_device_mesh_fan_hub_batches(W, n):
    """Batches of fan frames large enough (over 64k support candidates) for a star per
    16-lane group: a group records its full sets of 16 triangles for the rasterisation, up
    to 15 of them; the 3200-column fan's hub owns about 310 triangles, more than that, so
    those frames go to the host meshes. Every frame equals its solo solve."""
    from paper_1511_00758_amd import api
    left, right = scenes.fan_pair(W, 480, seed=78)
    prm = scenes.params_of(2)
    _note("fan batch", W, n)
    solo = api.Solver(W, 480, prm, device=DEV)(_dev(left), _dev(right))
    torch.cuda.synchronize()
    exp = (solo.D_f.cpu().numpy(), solo.C_f.cpu().numpy(), solo.mask.cpu().numpy())
    frames = [(_dev(left), _dev(right), prm) for _ in range(n)]
    outs, st = api.ManySolver(4, device=DEV)(frames, stats=True)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        got = tuple(t.cpu().numpy() for t in o)
        assert (got[0].view(np.uint32) == exp[0].view(np.uint32)).all(), i
        assert (got[1] == exp[1]).all() and (got[2] == exp[2]).all(), i
    assert st["mesh_fallback"] == (n if W > 2048 else 0)
