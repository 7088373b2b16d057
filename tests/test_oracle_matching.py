"""Pins of the oracle's support candidates and epipolar matcher."""
import numpy as np
import pytest

import oracle
import scenes


def _popcount(x):
    return bin(int(x)).count("1")


def _brute_decisions(cL, cR, cands, p, W):
    """Full cost volume over every pixel and disparity, then each candidate decided by
    enumeration (written independently of the oracle's matcher)."""
    H = cL.shape[0]
    nd = p.d_max - p.d_min + 1
    BIG = 10**9
    vol = np.full((H, W, nd), BIG, dtype=np.int64)       # left-to-right costs
    volr = np.full((H, W, nd), BIG, dtype=np.int64)      # right-to-left costs
    for v in range(H):
        for u in range(W):
            for k in range(nd):
                d = p.d_min + k
                if u - d >= p.rx:
                    vol[v, u, k] = _popcount(int(cL[v, u]) ^ int(cR[v, u - d]))
                if u + d <= W - 1 - p.rx:
                    volr[v, u, k] = _popcount(int(cR[v, u]) ^ int(cL[v, u + d]))
    out = []
    for (u, v) in cands:
        row = vol[v, u]
        adm = [k for k in range(nd) if row[k] < BIG]
        if not adm:
            continue
        best = min(row[k] for k in adm)
        kstar = min(k for k in adm if row[k] == best)
        if best >= p.t_hi:
            continue
        if p.uniqueness and any(row[k] < best + p.uniqueness for k in adm if abs(k - kstar) >= 2):
            continue
        ur = u - (p.d_min + kstar)
        rrow = volr[v, ur]
        adm2 = [k for k in range(nd) if rrow[k] < BIG]
        b2 = min(rrow[k] for k in adm2)
        k2 = min(k for k in adm2 if rrow[k] == b2)
        if abs(k2 - kstar) > p.lr_tol:
            continue
        out.append((u, v, float(p.d_min + kstar)))
    return out


@pytest.mark.parametrize("seed,cw,uniq,lr", [(0, 3, 1, 1), (1, 5, 0, 1), (2, 5, 2, 0), (3, 3, 1, 3)])
def test_matching_equals_brute_force_cost_volume(seed, cw, uniq, lr):
    W, H = 32, 24
    sc = scenes.slanted_plane(W, H, 6, 1, 0, g=10, seed=seed, sigma=3.0)
    p = oracle.Params(d_min=1, d_max=12, census_w=cw, census_h=cw, t_hi=cw * cw // 2,
                      uniqueness=uniq, lr_tol=lr)
    cL, valid = oracle.census(sc.left, cw, cw)
    cR, _ = oracle.census(sc.right, cw, cw)
    cands = [(u, v) for v in range(H) for u in range(W) if valid[v, u]]
    got = oracle.sparse_stereo(cL, cR, cands, p)
    ref = _brute_decisions(cL, cR, cands, p, W)
    assert got == ref
    assert len(got) > 0


def test_matching_random_images_brute_force():
    l, r = scenes.random_pair(28, 12, 5)
    p = oracle.Params(d_min=0, d_max=9, census_w=3, census_h=3, t_hi=9, uniqueness=1)
    cL, valid = oracle.census(l, 3, 3)
    cR, _ = oracle.census(r, 3, 3)
    cands = [(u, v) for v in range(12) for u in range(28) if valid[v, u]]
    assert oracle.sparse_stereo(cL, cR, cands, p) == _brute_decisions(cL, cR, cands, p, 28)


@pytest.mark.parametrize("d", [0, 7, 31])
def test_fronto_parallel_shift_recovers_disparity(d):
    """right(u, v) = left(u + d, v) exactly, so the true disparity costs 0. An accepted
    support must then cost 0 too; ties go to the smaller disparity and uniqueness
    rejects ties two or more apart, so the match is d or d - 1 (a locally ramp-like
    texture gives equal census words at neighbouring pixels); nearly all are d."""
    W, H = 160, 80
    sc = scenes.fronto_shift(W, H, d, seed=d)
    assert (sc.right[:, :W - d] == sc.left[:, d:]).all()
    p = oracle.Params(d_min=0, d_max=40, census_w=5, census_h=5, t_hi=6, grad_thr=8)
    cL, valid = oracle.census(sc.left, 5, 5)
    cR, _ = oracle.census(sc.right, 5, 5)
    om = oracle.high_gradient(sc.left, valid, p.grad_thr)
    cands = oracle.grid_candidates(W, H, 10, om)
    S = oracle.sparse_stereo(cL, cR, cands, p)
    eligible = [(u, v) for (u, v) in cands if u - d >= p.rx]
    S_elig = [s for s in S if s[0] - d >= p.rx]      # the true match is admissible
    for (u, v, dd) in S_elig:
        assert oracle.hamming(cL[v, u], cR[v, u - d]) == 0
        assert dd in (d, d - 1)
        assert oracle.hamming(cL[v, u], cR[v, u - int(dd)]) == 0
    exact = [s for s in S_elig if s[2] == d]
    assert len(exact) >= 0.9 * len(eligible)


def test_grid_candidates_layout():
    om = np.ones((30, 41), dtype=bool)
    c = oracle.grid_candidates(41, 30, 10, om)
    assert c[:5] == [(5, 5), (15, 5), (25, 5), (35, 5), (5, 15)]
    assert len(c) == 4 * 3
    om[15, 25] = False
    assert (25, 15) not in oracle.grid_candidates(41, 30, 10, om)
