"""GPU parity of the paper variants: FAST supports from spatial bins (Sec. III-A) and
multi-level cost evaluation (Sec. III-B), entry point by entry point and end to end,
bit for bit against the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _note(*a):
    print("[gpu-variants]", *a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _api():
    from paper_1511_00758_amd import api
    return api


def _images():
    rng = np.random.default_rng(21)
    out = [("random", rng.integers(0, 256, size=(61, 83), dtype=np.uint8)),
           ("quantised", np.linspace(0, 255, 4).astype(np.uint8)[rng.integers(0, 4, size=(47, 70))]),
           ("tiny_7x7", rng.integers(0, 256, size=(7, 7), dtype=np.uint8)),
           ("tiny_6x9", rng.integers(0, 256, size=(6, 9), dtype=np.uint8))]
    for cfg in (1, 2, 3):
        sc = scenes.make_scene(cfg, scenes.seed_of(cfg, 3))
        out.append((f"scene{cfg}", sc.left))
    return out


@pytest.mark.parametrize("name,img", _images(), ids=lambda x: x if isinstance(x, str) else "")
def test_fast_score_parity(name, img):
    _note("fast score", name, img.shape)
    api = _api()
    score, _, _ = api.fast_candidates(_dev(img), dict(scenes.params_of(2), fast_threshold=10, fast_bins_x=3,
                                                      fast_bins_y=2, fast_per_bin=4))
    torch.cuda.synchronize()
    assert (score.cpu().numpy().astype(np.int32) == oracle.fast_score(img)).all()


FAST_CASES = [(16, 12, 10, 25), (16, 12, 10, 1), (5, 12, 10, 2000), (30, 5, 7, 9), (0, 1, 1, 50),
              (40, 64, 3, 3)]


@pytest.mark.parametrize("t,bx,by,k", FAST_CASES)
def test_fast_candidates_parity(t, bx, by, k):
    api = _api()
    for name, img in _images():
        _note("fast candidates", name, t, bx, by, k)
        _, cand, n = api.fast_candidates(_dev(img), dict(scenes.params_of(2), fast_threshold=t, fast_bins_x=bx,
                                                         fast_bins_y=by, fast_per_bin=k))
        torch.cuda.synchronize()
        got = [tuple(int(x) for x in r) for r in cand[: int(n.item())].cpu().numpy()]
        assert got == oracle.fast_candidates(img, t, bx, by, k), name


def _low_density_words(rng, H, W, bits):
    rho = np.linspace(0.0, 0.5, H, dtype=np.float64)[:, None, None]
    on = rng.random((H, W, bits)) < rho
    weights = (np.uint64(1) << np.arange(bits, dtype=np.uint64))
    return (on.astype(np.uint64) * weights).sum(axis=2, dtype=np.uint64)


def _decode(keys, W, init, bad):
    out = {}
    for c, key in enumerate(keys.view(np.uint64).tolist()):
        if key != init:
            out[c] = (key & 0xffffffff) % W, (key & 0xffffffff) // W, 255 - (key >> 32) if bad else key >> 32
    return out


def _cells(cells):
    Wc = len(cells[0])
    return {cy * Wc + cx: (c.u, c.v, c.cost) for cy, row in enumerate(cells) for cx, c in enumerate(row)
            if c.set}


@pytest.mark.parametrize("levels", [3, 5])
@pytest.mark.parametrize("size,sz", [((320, 240), 8), ((333, 487), 1), ((640, 480), 32)])
def test_validate_levels_parity(levels, size, sz):
    api = _api()
    W, H = size
    _note("validate levels", levels, size, sz)
    rng = np.random.default_rng(levels * 100 + sz)
    prm = dict(scenes.params_of(2), levels=levels)
    p = oracle.Params.from_dict(prm)
    cL = _low_density_words(rng, H, W, 48)
    cR = _low_density_words(rng, H, W, 48)
    omega = rng.random((H, W)) < 0.7
    D_it = rng.uniform(-2.5, p.d_max + 3.0, size=(H, W)).astype(np.float32)
    D_it[rng.random((H, W)) < 0.1] = np.nan
    D_f0 = rng.uniform(0, 50, size=(H, W)).astype(np.float32)
    C_f0 = rng.integers(0, p.t_hi + 1, size=(H, W)).astype(np.uint8)
    C_exp = oracle.cost_evaluation(cL, cR, omega, D_it, p)
    D_exp, Cf_exp = D_f0.copy(), C_f0.copy()
    Cg, Cb = oracle.disparity_refinement(D_it, C_exp, D_exp, Cf_exp, p, sz)
    D_f, C_f = _dev(D_f0), _dev(C_f0)
    C_it, g, b = api.validate(_dev(cL.view(np.int64)), _dev(cR.view(np.int64)), _dev(omega.astype(np.uint8)),
                              _dev(D_it), prm, sz, D_f, C_f)
    torch.cuda.synchronize()
    assert (C_it.cpu().numpy() == C_exp).all()
    assert (C_f.cpu().numpy() == Cf_exp).all()
    assert (D_f.cpu().numpy().view(np.uint32) == D_exp.view(np.uint32)).all()
    assert _decode(g.cpu().numpy(), W, p.t_lo << 32, False) == _cells(Cg)
    assert _decode(b.cpu().numpy(), W, (255 - p.t_hi) << 32, True) == _cells(Cb)


def _solve_gpu(sc, params):
    api = _api()
    H, W = sc.left.shape
    s = api.Solver(W, H, params, device=DEV)
    r = s(_dev(sc.left), _dev(sc.right), stats=True, timing=True)
    torch.cuda.synchronize()
    return r.D_f.cpu().numpy(), r.C_f.cpu().numpy(), r.mask.cpu().numpy(), r.stats


VARIANTS = [(1, 1, 0), (1, 1, 1), (1, 3, 1), (2, 1, 1), (2, 3, 0), (2, 5, 1), (3, 3, 1)]


@pytest.mark.parametrize("cfg,levels,mode", VARIANTS)
def test_solve_variants_parity(cfg, levels, mode):
    _note("solve variant", cfg, levels, mode)
    sc = scenes.make_scene(cfg, scenes.seed_of(cfg, 2))
    prm = dict(sc.params, levels=levels, support_mode=mode)
    p = oracle.Params.from_dict(prm)
    tr = oracle.solve(sc.left, sc.right, p, trace=True)
    D_f, C_f, mask, st = _solve_gpu(sc, prm)
    assert st["n_support"] == [len(it["S"]) for it in tr["iters"]]
    assert (C_f == tr["C_f"]).all()
    assert (mask.astype(bool) == tr["mask"]).all()
    assert (D_f.view(np.uint32) == tr["D_f"].view(np.uint32)).all()
    if mode == 1:
        assert st["stage_launches"]["fast"] == 2
    else:
        assert st["stage_launches"]["fast"] == 0
