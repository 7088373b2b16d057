"""Pins of the oracle's FAST keypoints (Sec. III-A) and multi-level cost evaluation
(Sec. III-B), independent of the formulas they check: geometry of the circle, hand-derived
scores, a run-length brute force of the segment test, an explicit-loop non-maximum
suppression and bin selection, and per-pixel loops over disparity levels."""
import math

import numpy as np
import pytest

import oracle
from oracle.params import Params


# ----------------------------------------------------------------------------------
# circle
# ----------------------------------------------------------------------------------
def test_circle_is_the_radius_3_bresenham_ring_in_clockwise_order():
    pts = oracle.CIRCLE
    assert len(pts) == 16 and len(set(pts)) == 16
    for dx, dy in pts:
        assert 2.8 <= math.hypot(dx, dy) <= 3.2
    # clockwise from straight up, with image rows growing downwards: the angle measured
    # from "up" towards "right" increases strictly
    ang = [math.atan2(dx, -dy) % (2 * math.pi) for dx, dy in pts]
    assert ang[0] == 0.0 and all(a < b for a, b in zip(ang, ang[1:]))
    # contiguous: consecutive ring pixels are 8-neighbours of each other
    for k in range(16):
        (x0, y0), (x1, y1) = pts[k], pts[(k + 1) % 16]
        assert max(abs(x1 - x0), abs(y1 - y0)) == 1


# ----------------------------------------------------------------------------------
# scores: hand-derived cases
# ----------------------------------------------------------------------------------
def test_isolated_bright_pixel_scores_its_contrast():
    img = np.full((15, 15), 50, np.uint8)
    img[7, 7] = 200
    s = oracle.fast_score(img)
    assert s[7, 7] == 150          # every circle pixel is darker by exactly 150
    assert oracle.keypoints(s, 149)[7, 7] and not oracle.keypoints(s, 150)[7, 7]


def test_straight_edge_is_not_a_corner():
    img = np.full((15, 15), 50, np.uint8)
    img[:, 8:] = 200               # p = (7, 7) on the dark side, right next to the edge
    s = oracle.fast_score(img)
    # bright circle pixels are those with dx >= 1: 7 of them, fewer than 9 in a row;
    # every other circle pixel equals I(p), so no arc of 9 is strictly brighter or darker
    assert s[7, 7] == 0


def test_corner_of_a_dark_quadrant_scores_the_contrast():
    img = np.full((15, 15), 200, np.uint8)
    img[:8, :8] = 50               # dark quadrant u <= 7, v <= 7; p = (7, 7) its corner
    s = oracle.fast_score(img)
    # dark circle pixels are those with dx <= 0 and dy <= 0: (0,-3), (-3,0), (-3,-1),
    # (-2,-2), (-1,-3); the other 11 form one run of bright pixels, each +150
    assert s[7, 7] == 150


def test_border_pixels_score_zero():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, size=(12, 13), dtype=np.uint8)
    s = oracle.fast_score(img)
    assert (s[:3] == 0).all() and (s[-3:] == 0).all() and (s[:, :3] == 0).all() and (s[:, -3:] == 0).all()
    assert (oracle.fast_score(img[:6, :]) == 0).all()


# ----------------------------------------------------------------------------------
# scores: run-length brute force of the segment test
# ----------------------------------------------------------------------------------
def _segment_test(img, u, v, t):
    c = int(img[v, u])
    ring = [int(img[v + dy, u + dx]) - c for dx, dy in oracle.CIRCLE]
    for sign in (1, -1):
        run = best = 0
        for x in ring + ring:       # the ring read twice covers every wrap-around run
            run = run + 1 if sign * x > t else 0
            best = max(best, run)
        if min(best, 16) >= 9:
            return True
    return False


@pytest.mark.parametrize("seed,levels", [(0, 256), (1, 4), (2, 3), (3, 256)])
def test_score_is_the_largest_passing_threshold_plus_one(seed, levels):
    rng = np.random.default_rng(seed)
    vals = np.linspace(0, 255, levels).astype(np.uint8)
    img = vals[rng.integers(0, levels, size=(11, 12))]
    s = oracle.fast_score(img)
    H, W = img.shape
    for v in range(3, H - 3):
        for u in range(3, W - 3):
            passing = [t for t in range(0, 256) if _segment_test(img, u, v, t)]
            expect = max(passing) + 1 if passing else 0
            assert s[v, u] == expect, (u, v)


# ----------------------------------------------------------------------------------
# non-maximum suppression and bins
# ----------------------------------------------------------------------------------
def _nms_loops(score, t):
    H, W = score.shape
    out = np.zeros((H, W), bool)
    for v in range(H):
        for u in range(W):
            if score[v, u] <= t:
                continue
            ok = True
            for dv in (-1, 0, 1):
                for du in (-1, 0, 1):
                    q = (v + dv, u + du)
                    if (dv, du) == (0, 0) or not (0 <= q[0] < H and 0 <= q[1] < W):
                        continue
                    sq = score[q]
                    if (q[0], q[1]) < (v, u):      # earlier in raster order
                        ok &= sq < score[v, u]
                    else:
                        ok &= sq <= score[v, u]
            out[v, u] = ok
    return out


@pytest.mark.parametrize("seed", range(3))
def test_non_maximum_suppression_matches_explicit_loops(seed):
    rng = np.random.default_rng(10 + seed)
    score = rng.integers(0, 6, size=(14, 17))       # many equal neighbours
    for t in (0, 2, 4):
        assert (oracle.keypoints(score, t) == _nms_loops(score, t)).all()


def test_equal_plateau_keeps_only_its_first_pixel():
    score = np.zeros((6, 6), np.int64)
    score[2:4, 1:5] = 7
    kp = oracle.keypoints(score, 3)
    assert kp.sum() == 1 and kp[2, 1]


@pytest.mark.parametrize("per_bin", [1, 3, 50])
def test_bin_selection_matches_explicit_sort(per_bin):
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(40, 57), dtype=np.uint8)
    t, bx, by = 20, 4, 3
    got = oracle.fast_candidates(img, t, bx, by, per_bin)
    kp = _nms_loops(oracle.fast_score(img), t)
    s = oracle.fast_score(img)
    H, W = img.shape
    expect = []
    for b_y in range(by):
        for b_x in range(bx):
            members = [(v, u) for v in range(H) for u in range(W)
                       if kp[v, u] and u * bx // W == b_x and v * by // H == b_y]
            members.sort(key=lambda q: (-s[q], q))
            expect.extend((u, v) for (v, u) in sorted(members[:per_bin]))
    assert got == expect
    if per_bin == 50:              # no bin is full: every keypoint is a candidate
        assert len(got) == int(kp.sum())


def test_bins_cover_the_image_with_widths_differing_by_at_most_one():
    W, H, bx, by = 640, 480, 12, 10
    widths = np.bincount([u * bx // W for u in range(W)], minlength=bx)
    heights = np.bincount([v * by // H for v in range(H)], minlength=by)
    assert widths.sum() == W and widths.max() - widths.min() <= 1
    assert heights.sum() == H and heights.max() - heights.min() <= 1


# ----------------------------------------------------------------------------------
# multi-level cost evaluation
# ----------------------------------------------------------------------------------
def _cost_loops(cL, cR, omega, D, p):
    H, W = cL.shape
    C = np.full((H, W), 0xFF, np.uint8)
    k = (p.levels - 1) // 2
    for v in range(H):
        for u in range(W):
            if not omega[v, u] or not np.isfinite(D[v, u]):
                continue
            d = math.floor(float(np.float32(D[v, u]) + np.float32(0.5)))
            if not (p.d_min <= d <= p.d_max and u - d >= p.rx):
                continue
            best = 255
            for dl in range(d - k, d + k + 1):
                if p.d_min <= dl <= p.d_max and u - dl >= p.rx:
                    best = min(best, bin(int(cL[v, u]) ^ int(cR[v, u - dl])).count("1"))
            C[v, u] = best
    return C


@pytest.mark.parametrize("levels", [1, 3, 5])
def test_multilevel_cost_matches_loops(levels):
    rng = np.random.default_rng(levels)
    H, W = 9, 40
    cL = rng.integers(0, 2 ** 24, size=(H, W), dtype=np.int64).astype(np.uint64)
    cR = rng.integers(0, 2 ** 24, size=(H, W), dtype=np.int64).astype(np.uint64)
    omega = rng.random((H, W)) < 0.8
    D = rng.uniform(-1.0, 20.0, size=(H, W)).astype(np.float32)
    D[rng.random((H, W)) < 0.1] = np.nan
    p = Params(d_min=1, d_max=15, census_w=5, census_h=5, levels=levels)
    assert (oracle.cost_evaluation(cL, cR, omega, D, p) == _cost_loops(cL, cR, omega, D, p)).all()


def test_more_levels_never_raise_the_cost_and_keep_the_evaluated_set():
    rng = np.random.default_rng(9)
    H, W = 12, 60
    cL = rng.integers(0, 2 ** 48, size=(H, W), dtype=np.int64).astype(np.uint64)
    cR = rng.integers(0, 2 ** 48, size=(H, W), dtype=np.int64).astype(np.uint64)
    omega = np.ones((H, W), bool)
    D = rng.uniform(0, 30, size=(H, W)).astype(np.float32)
    prev = None
    for L in (1, 3, 5):
        C = oracle.cost_evaluation(cL, cR, omega, D, Params(d_max=31, census_w=7, census_h=7, levels=L))
        if prev is not None:
            assert ((C == 0xFF) == (prev == 0xFF)).all()
            assert (C <= prev).all()
        prev = C


def test_plane_off_by_one_level_is_validated_with_three_levels():
    """Right image = left shifted by s: with D_it = s + 1 everywhere, one level sees
    mismatching words, three levels find the true column at cost 0."""
    rng = np.random.default_rng(4)
    H, W, s = 20, 80, 6
    left = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    right = np.zeros_like(left)
    right[:, : W - s] = left[:, s:]
    cL, valid = oracle.census(left, 5, 5)
    cR, _ = oracle.census(right, 5, 5)
    omega = valid.copy()
    omega[:, : s + 2] = False
    omega[:, W - s - 2:] = False
    D = np.full((H, W), s + 1, np.float32)
    one = oracle.cost_evaluation(cL, cR, omega, D, Params(d_max=20, levels=1))
    three = oracle.cost_evaluation(cL, cR, omega, D, Params(d_max=20, levels=3))
    ev = three != 0xFF
    assert ev.sum() > 500
    assert (three[ev] == 0).all() and (one[ev] > 0).mean() > 0.9


def test_fast_supported_solve_recovers_the_four_plane_scene():
    """Alg. 1 with FAST supports (and with three levels) on the 320x240 scene: most
    validated pixels lie within 3 px of the ground truth (a guard against gross errors
    in the detector's use, not a parity pin)."""
    import scenes
    sc = scenes.make_scene(1, scenes.seed_of(1, 0))
    for levels in (1, 3):
        prm = dict(sc.params, support_mode=1, levels=levels)
        r = oracle.solve(sc.left, sc.right, Params.from_dict(prm))
        ok = r["mask"] & np.isfinite(sc.disp)
        assert ok.mean() > 0.4
        assert (np.abs(r["D_f"][ok] - sc.disp[ok]) <= 3).mean() > 0.85
