"""Host-side checks of the C ABI that need no GPU: the library loads and exports every
declared entry point, the host triangulation equals the oracle's, and invalid
arguments are rejected before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1511_00758_amd import _lib
from paper_1511_00758_amd.api import SUPPORT_DTYPE, triangulate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stereomesh.h")

lib_missing = not os.path.exists(_lib.LIB_PATH)
pytestmark = pytest.mark.skipif(lib_missing, reason="libstereomesh.so not built (run __graft_entry__.build())")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = _lib.load()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert b"gfx950" in L.sm_version()


def _S(points, d=None):
    S = np.zeros(len(points), dtype=SUPPORT_DTYPE)
    for i, (u, v) in enumerate(points):
        S[i] = (u, v, 0.0 if d is None else d[i])
    return S


def _oracle_tris(S, W):
    return oracle.triangulate([(int(s["u"]), int(s["v"]), float(s["d"])) for s in S], W)


@pytest.mark.parametrize("seed,n,span", [(0, 50, 30), (1, 400, 200), (2, 300, 12), (3, 1000, 4000),
                                         (4, 60, 5)])
def test_triangulate_equals_oracle_random(seed, n, span):
    rng = np.random.default_rng(seed)
    pts = [(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)]  # with dups
    S = _S(pts)
    got = [tuple(t) for t in triangulate(S)]
    assert got == _oracle_tris(S, 8192)


@pytest.mark.parametrize("nx,ny,g", [(64, 48, 10), (7, 5, 3), (1, 9, 4), (30, 2, 6)])
def test_triangulate_equals_oracle_grid(nx, ny, g):
    pts = [(g // 2 + i * g, g // 2 + j * g) for j in range(ny) for i in range(nx)]
    rng = np.random.default_rng(nx * ny)
    keep = rng.random(len(pts)) > 0.15
    S = _S([p for p, k in zip(pts, keep) if k])
    got = [tuple(t) for t in triangulate(S)]
    assert got == _oracle_tris(S, 8192)


def test_triangulate_incremental_batches_equal_rebuild():
    """Inserting supports in any order (as the solver does across iterations) gives the
    unique triangulation."""
    rng = np.random.default_rng(9)
    pts = list({(int(rng.integers(0, 300)), int(rng.integers(0, 200))) for _ in range(700)})
    grid = [(5 + 10 * i, 5 + 10 * j) for j in range(20) for i in range(30)]
    S = _S(grid + [p for p in pts if p not in set(grid)])
    got = [tuple(t) for t in triangulate(S)]
    assert got == _oracle_tris(S, 8192)


def test_triangulate_degenerate_and_errors():
    assert triangulate(_S([])).shape == (0, 3)
    assert triangulate(_S([(1, 1), (3, 3)])).shape == (0, 3)
    assert triangulate(_S([(i, 2 * i) for i in range(9)])).shape == (0, 3)
    S = _S([(0, 0), (10, 0), (0, 10)])
    L = _lib.load()
    arr = np.zeros(1, dtype=np.int32)
    nt = ctypes.c_int32(0)
    st = L.sm_triangulate(S.ctypes.data, 3, arr.ctypes.data, 0, ctypes.byref(nt))
    assert st == _lib.SM_ERR_CAPACITY and nt.value == 1
    bad = _S([(9000, 0), (0, 1), (1, 0)])
    with pytest.raises(_lib.StereoMeshError):
        triangulate(bad)


def _params(**kw):
    d = dict(d_min=0, d_max=63, census_w=5, census_h=5, support_step=10, n_iters=1, t_hi=8,
             t_lo=4, grad_thr=16, lr_tol=1, uniqueness=1, sz_occ0=32)
    d.update(kw)
    return _lib.make_params(d)


FAKE = 0x10000  # never dereferenced: every call below fails argument checks first


@pytest.mark.parametrize("kw", [dict(d_min=5, d_max=4), dict(d_max=256), dict(census_w=4),
                                dict(census_w=9, census_h=9), dict(n_iters=0), dict(n_iters=9),
                                dict(t_lo=9), dict(t_hi=65), dict(support_step=0),
                                dict(sz_occ0=0), dict(grad_thr=-1), dict(uniqueness=-1),
                                dict(levels=2), dict(levels=0), dict(levels=7), dict(support_mode=2),
                                dict(support_mode=1, fast_threshold=255),
                                dict(support_mode=1, fast_bins_x=0), dict(support_mode=1, fast_bins_y=1025),
                                dict(support_mode=1, fast_per_bin=0),
                                dict(support_mode=1, fast_bins_x=1024, fast_bins_y=1024, fast_per_bin=8)])
def test_bad_params_rejected(kw):
    L = _lib.load()
    p = _params(**kw)
    assert L.sm_solve_workspace_bytes(64, 48, p) == 0
    st = L.sm_solve(FAKE, FAKE, 64, 48, 64, p, FAKE, 1 << 30, FAKE, FAKE, FAKE, None, None)
    assert st == _lib.SM_ERR_ARG
    assert L.sm_last_error()


def test_bad_sizes_and_pointers_rejected():
    L = _lib.load()
    p = _params()
    assert L.sm_census(FAKE, 2, 48, 2, 5, 5, 0, FAKE, None, None) == _lib.SM_ERR_ARG
    assert L.sm_census(FAKE, 64, 48, 32, 5, 5, 0, FAKE, None, None) == _lib.SM_ERR_ARG  # stride < W
    assert L.sm_census(None, 64, 48, 64, 5, 5, 0, FAKE, None, None) == _lib.SM_ERR_ARG
    assert L.sm_census(FAKE, 9000, 48, 9000, 5, 5, 0, FAKE, None, None) == _lib.SM_ERR_ARG
    # grid mode needs omega; capacity must cover every candidate
    n = ctypes.c_int32(0)
    assert L.sm_match_support(FAKE, FAKE, None, 64, 48, None, 0, p, FAKE, 100, FAKE, None) == _lib.SM_ERR_ARG
    assert L.sm_grid_candidates(64, 48, 10) == 6 * 5
    assert L.sm_match_support(FAKE, FAKE, FAKE, 64, 48, None, 0, p, FAKE, 29, FAKE, None) == _lib.SM_ERR_CAPACITY
    assert L.sm_cells(64, 48, 32) == 4 and L.sm_cells(640, 480, 8) == 4800
    assert L.sm_resample(FAKE, FAKE, FAKE, FAKE, FAKE, 64, 48, 32, p, None, 0, FAKE, FAKE, 7, FAKE,
                         None) == _lib.SM_ERR_CAPACITY
    assert L.sm_validate(FAKE, FAKE, FAKE, FAKE, 64, 48, p, 0, None, FAKE, FAKE, FAKE, FAKE,
                         None) == _lib.SM_ERR_ARG
    ws = L.sm_solve_workspace_bytes(64, 48, p)
    assert ws > 64 * 48 * 22
    assert L.sm_solve(FAKE, FAKE, 64, 48, 64, p, FAKE, ws - 1, FAKE, FAKE, FAKE, None, None) == _lib.SM_ERR_CAPACITY
    assert L.sm_solve(FAKE, FAKE, 64, 48, 64, p, FAKE + 8, ws, FAKE, FAKE, FAKE, None, None) == _lib.SM_ERR_ARG


def test_fast_candidates_rejects_bad_arguments():
    L = _lib.load()
    p = _params(fast_bins_x=4, fast_bins_y=3, fast_per_bin=5)
    n = 4 * 3 * 5
    ok = L.sm_fast_candidates
    assert ok(FAKE, 64, 48, 64, p, FAKE, FAKE, n - 1, FAKE, None) == _lib.SM_ERR_CAPACITY
    assert ok(FAKE, 64, 48, 63, p, FAKE, FAKE, n, FAKE, None) == _lib.SM_ERR_ARG      # stride < W
    assert ok(None, 64, 48, 64, p, FAKE, FAKE, n, FAKE, None) == _lib.SM_ERR_ARG
    assert ok(FAKE, 64, 48, 64, p, None, FAKE, n, FAKE, None) == _lib.SM_ERR_ARG      # score scratch
    assert ok(FAKE, 2, 48, 64, p, FAKE, FAKE, n, FAKE, None) == _lib.SM_ERR_ARG
    assert ok(FAKE, 64, 48, 64, _params(fast_threshold=300), FAKE, FAKE, n, FAKE, None) == _lib.SM_ERR_ARG
    assert L.sm_last_error()


def test_fast_mode_workspace_holds_the_bin_slots_and_scores():
    L = _lib.load()
    # (host meshes on both sides: grid frames otherwise also hold the device mesh buffers)
    grid = L.sm_solve_workspace_bytes(640, 480, _params(host_mesh=1))
    fast = L.sm_solve_workspace_bytes(640, 480, _params(support_mode=1, fast_per_bin=400, host_mesh=1))
    # 12 x 10 bins x 400 slots of 8 bytes (vs 3072 grid slots) plus 1 B/px of scores
    assert fast - grid >= 640 * 480 + (120 * 400 - 3072) * 8
