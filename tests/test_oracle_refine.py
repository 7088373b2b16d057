"""Pins of the oracle's CostEvaluation (Alg. 2), DisparityRefinement (Alg. 3),
SupportResampling (Alg. 4) and the iteration of Alg. 1."""
import numpy as np
import pytest

import oracle
import scenes
from oracle.refine import NOT_EVALUATED


def _popcount(x):
    return bin(int(x)).count("1")


@pytest.fixture(scope="module")
def c2_trace():
    sc = scenes.make_scene(2, scenes.seed_of(2, 1))
    p = oracle.Params.from_dict(sc.params)
    return sc, p, oracle.solve(sc.left, sc.right, p, trace=True)


def test_cost_evaluation_equals_brute_force(c2_trace):
    sc, p, r = c2_trace
    cL, cR, om = r["cL"], r["cR"], r["omega"]
    it = r["iters"][0]
    D, C = it["D_it"], it["C_it"]
    H, W = D.shape
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(4000):
        u, v = int(rng.integers(0, W)), int(rng.integers(0, H))
        exp = NOT_EVALUATED
        if om[v, u] and np.isfinite(D[v, u]):
            d = int(np.floor(np.float32(D[v, u]) + np.float32(0.5)))
            if p.d_min <= d <= p.d_max and u - d >= p.rx:
                exp = _popcount(int(cL[v, u]) ^ int(cR[v, u - d]))
                checked += 1
        assert C[v, u] == exp
    assert checked > 1000


def test_cost_rounding_boundary():
    """floor(D + 0.5) in float32: 2.5 -> 3, 2.4999998 -> 2, -0.5 -> 0 (then admissible)."""
    cL = np.zeros((1, 12), np.uint64)
    cR = np.arange(12, dtype=np.uint64).reshape(1, 12)
    om = np.ones((1, 12), bool)
    p = oracle.Params(d_min=0, d_max=5, census_w=1, census_h=1)
    D = np.full((1, 12), np.nan, np.float32)
    D[0, 8] = 2.5
    D[0, 9] = np.nextafter(np.float32(2.5), np.float32(0))
    D[0, 10] = -0.5
    D[0, 11] = 5.6     # rounds to 6 > d_max: not evaluated
    C = oracle.cost_evaluation(cL, cR, om, D, p)
    assert C[0, 8] == _popcount(8 - 3)
    assert C[0, 9] == _popcount(9 - 2)
    assert C[0, 10] == _popcount(10)
    assert C[0, 11] == NOT_EVALUATED and C[0, 0] == NOT_EVALUATED


def test_fronto_parallel_validation_is_exact():
    """Pure shift by d, no noise: on every triangle whose three supports carry d, the
    interpolated disparity is exactly d, every evaluated pixel costs 0 and every
    Omega_I pixel with an admissible column passes validation."""
    from oracle.interp import owned_pixels
    W, H, d = 160, 96, 9
    sc = scenes.fronto_shift(W, H, d, seed=4)
    p = oracle.Params(d_min=0, d_max=31, census_w=5, census_h=5, t_hi=6, t_lo=3, grad_thr=8,
                      n_iters=2)
    r = oracle.solve(sc.left, sc.right, p, trace=True)
    for it in r["iters"]:
        S = it["S"]
        good = [s for s in S if s[0] - d >= p.rx]
        assert all(s[2] == d or s[2] == d - 1 for s in good)
    it = r["iters"][0]
    S, D, C = it["S"], it["D_it"], it["C_it"]
    exact_tris = [t for t in it["tris"] if all(S[i][2] == d for i in t)]
    assert len(exact_tris) > 0.8 * len(it["tris"])
    n = 0
    for t in exact_tris:
        us, vs = owned_pixels(S, t, W, H)
        assert (D[vs, us] == d).all()
        sel = r["omega"][vs, us] & (us - d >= p.rx)
        assert (C[vs[sel], us[sel]] == 0).all()
        assert (it["C_f"][vs[sel], us[sel]] < p.t_hi).all()
        n += sel.sum()
    assert n > 0.5 * r["omega"].sum()


def _cells_by_sort(C_it, D_it, p, sz):
    """Per-cell winners by sorting (cost, raster index) -- independent of the oracle's
    sequential loop; must agree with the first-in-raster-order rule."""
    H, W = C_it.shape
    vs, us = np.nonzero(C_it != NOT_EVALUATED)
    c = C_it[vs, us].astype(np.int64)
    idx = vs * W + us
    cell = (vs // sz) * (-(-W // sz)) + us // sz
    best_g, best_b = {}, {}
    for k in np.lexsort((idx, c)):                       # ascending cost, then index
        if c[k] < p.t_lo and cell[k] not in best_g:
            best_g[cell[k]] = (us[k], vs[k], c[k])
    for k in np.lexsort((idx, -c)):                      # descending cost, then index
        if c[k] > p.t_hi and cell[k] not in best_b:
            best_b[cell[k]] = (us[k], vs[k], c[k])
    return best_g, best_b


def test_refinement_cells_equal_sorted_winners(c2_trace):
    sc, p, r = c2_trace
    for it in r["iters"]:
        sz = it["sz_occ"]
        g, b = _cells_by_sort(it["C_it"], it["D_it"], p, sz)
        Wc = -(-sc.left.shape[1] // sz)
        for cy, row in enumerate(it["Cg"]):
            for cx, cell in enumerate(row):
                key = cy * Wc + cx
                assert cell.set == (key in g)
                if cell.set:
                    assert (cell.u, cell.v, cell.cost) == tuple(int(x) for x in g[key])
                    assert cell.d == float(it["D_it"][cell.v, cell.u])
        for cy, row in enumerate(it["Cb"]):
            for cx, cell in enumerate(row):
                key = cy * Wc + cx
                assert cell.set == (key in b)
                if cell.set:
                    assert (cell.u, cell.v, cell.cost) == tuple(int(x) for x in b[key])


def test_final_cost_never_increases(c2_trace):
    """DisparityRefinement keeps the least cost per pixel: C_f is non-increasing over
    the iterations and D_f only changes where C_f strictly drops."""
    sc, p, r = c2_trace
    prev_C = np.full(sc.left.shape, p.t_hi, np.uint8)
    prev_D = np.zeros(sc.left.shape, np.float32)
    for it in r["iters"]:
        C, D = it["C_f"], it["D_f"]
        assert (C <= prev_C).all()
        same = C == prev_C
        assert (D[same] == prev_D[same]).all()
        prev_C, prev_D = C, D
    assert (r["mask"] == (r["omega"] & (r["C_f"] < p.t_hi))).all()


def test_resampling_invariants(c2_trace):
    sc, p, r = c2_trace
    its = r["iters"]
    assert [it["sz_occ"] for it in its] == [32, 16, 8]
    for a, b in zip(its, its[1:]):
        Sa, Sb = a["S"], b["S"]
        assert Sb[:len(Sa)] == Sa                              # S_it is a prefix of S_it+1
        new = Sb[len(Sa):]
        cells = len(a["Cg"]) * len(a["Cg"][0])
        assert len(new) <= 2 * cells
        keys = [(s[0], s[1]) for s in Sb]
        assert len(set(keys)) == len(keys)
        C = a["C_it"]
        for (u, v, d) in a["confident"]:
            assert C[v, u] < p.t_lo and d == float(a["D_it"][v, u])
        for (u, v) in a["X"]:
            assert C[v, u] != NOT_EVALUATED and C[v, u] > p.t_hi
        assert len(a["X"]) == sum(c.set for row in a["Cb"] for c in row)
        # matched supports are exactly the matcher's verdicts on X
        assert a["matched"] == oracle.sparse_stereo(r["cL"], r["cR"], a["X"], p)


def test_occupancy_schedule():
    p = oracle.Params(sz_occ0=32)
    assert [oracle.occupancy_size(p, i) for i in range(1, 9)] == [32, 16, 8, 4, 2, 1, 1, 1]
    p = oracle.Params(sz_occ0=24)
    assert [oracle.occupancy_size(p, i) for i in range(1, 7)] == [24, 12, 6, 3, 1, 1]


def test_single_iteration_does_not_resample():
    sc = scenes.make_scene(1, scenes.seed_of(1, 2))
    p = oracle.Params.from_dict(sc.params)
    r = oracle.solve(sc.left, sc.right, p, trace=True)
    assert len(r["iters"]) == 1 and "X" not in r["iters"][0]


def test_accuracy_against_ground_truth():
    """Context, and a guard against gross mistakes (a flipped disparity sign, a shifted
    window): on the 4-plane workload most validated, visible pixels lie within 3 px of
    the synthetic truth."""
    sc = scenes.make_scene(1, scenes.seed_of(1, 0))
    p = oracle.Params.from_dict(sc.params)
    r = oracle.solve(sc.left, sc.right, p)
    m = r["mask"] & sc.visible
    assert m.sum() > 0.3 * m.size
    err = np.abs(r["D_f"][m] - sc.disp[m])
    assert (err < 3).mean() > 0.9


def test_constant_image_is_degenerate_not_error():
    img = np.full((60, 80), 100, np.uint8)
    p = oracle.Params(n_iters=2)
    r = oracle.solve(img, img, p)
    assert not r["mask"].any() and (r["D_f"] == 0).all() and (r["C_f"] == p.t_hi).all()
