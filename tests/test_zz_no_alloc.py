"""GPU: sm_solve_noalloc (the allocation-free solve on the library's per-device
workspace) returns, call after call, exactly what sm_solve returns for the same frame:
a large frame, then smaller ones in the same workspace (whose contents the earlier call
left), then a frame without supports; frames above the workspace limit are refused
before any work."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-noalloc]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _noalloc(l, r, prm):
    from paper_1511_00758_amd import _lib
    L = _lib.load()
    H, W = l.shape
    left, right = _dev(l), _dev(r)
    D = torch.full((H, W), 7.0, dtype=torch.float32, device=DEV)
    C = torch.full((H, W), 99, dtype=torch.uint8, device=DEV)
    M = torch.full((H, W), 3, dtype=torch.uint8, device=DEV)
    st = _lib.SmStats()
    torch.cuda.synchronize()
    status = L.sm_solve_noalloc(left.data_ptr(), right.data_ptr(), W, H, W, _lib.make_params(prm),
                                D.data_ptr(), C.data_ptr(), M.data_ptr(), ctypes.byref(st),
                                torch.cuda.current_stream().cuda_stream)
    _lib.check(status)
    return D.cpu().numpy(), C.cpu().numpy(), M.cpu().numpy(), st


def _solve(l, r, prm):
    from paper_1511_00758_amd import api
    H, W = l.shape
    res = api.Solver(W, H, prm, device=DEV)(_dev(l), _dev(r), stats=True)
    torch.cuda.synchronize()
    return res.D_f.cpu().numpy(), res.C_f.cpu().numpy(), res.mask.cpu().numpy(), res.stats


def _frames():
    big = scenes.make_rect_scene(1280, 720, seed=6100, dlo=2.0, dhi=240.0)
    vga = scenes.make_scene(2, scenes.seed_of(2, 60))
    qvga = scenes.make_scene(1, scenes.seed_of(1, 60))
    flat = np.full((120, 160), 90, np.uint8)
    return [("1280x720 d0-255", big.left, big.right, scenes.params_of(5)),
            ("640x480", vga.left, vga.right, vga.params),
            ("320x240", qvga.left, qvga.right, qvga.params),
            ("flat 160x120", flat, flat.copy(), scenes.params_of(2))]


def test_noalloc_equals_sm_solve_call_after_call():
    frames = _frames()
    for rep in range(2):
        for name, l, r, prm in frames:   # every call after the first reuses a dirtier workspace
            _note("rep", rep, name)
            D, C, M, st = _noalloc(l, r, prm)
            sD, sC, sM, sst = _solve(l, r, prm)
            assert (D.view(np.uint32) == sD.view(np.uint32)).all(), name
            assert (C == sC).all(), name
            assert (M == sM).all(), name
            assert int(st.n_valid) == sst["n_valid"] == int(sM.sum()), name
            n = prm["n_iters"]
            assert list(st.n_support[:n]) == sst["n_support"], name
            assert list(st.n_tris[:n]) == sst["n_tris"], name


def test_noalloc_refuses_before_work():
    from paper_1511_00758_amd import _lib
    L = _lib.load()
    prm = scenes.params_of(5)
    W, H = 2560, 1440
    assert L.sm_solve_workspace_bytes(W, H, _lib.make_params(prm)) > _lib.NOALLOC_MAX_BYTES
    img = torch.zeros((H, W), dtype=torch.uint8, device=DEV)
    out = torch.zeros((H, W), dtype=torch.float32, device=DEV)
    u8 = torch.zeros((H, W), dtype=torch.uint8, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    st = L.sm_solve_noalloc(img.data_ptr(), img.data_ptr(), W, H, W, _lib.make_params(prm), out.data_ptr(),
                            u8.data_ptr(), u8.data_ptr(), None, s)
    assert st == _lib.SM_ERR_CAPACITY and b"sm_solve_noalloc" in L.sm_last_error()
    for over in (dict(host_mesh=1),):
        st = L.sm_solve_noalloc(img.data_ptr(), img.data_ptr(), 320, 240, 320,
                                _lib.make_params(dict(scenes.params_of(1), **over)), out.data_ptr(),
                                u8.data_ptr(), u8.data_ptr(), None, s)
        assert st == _lib.SM_ERR_ARG
    torch.cuda.synchronize()
    assert int(out.abs().sum().item()) == 0   # nothing was enqueued
