"""Pins of the oracle's disparity planes, pixel ownership and interpolation."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes
from oracle.interp import owned_pixels


def _exact_plane(S, t):
    """Rational plane through the three supports: returns (A, B, C) with d = A u + B v + C."""
    (u0, v0, d0), (u1, v1, d1), (u2, v2, d2) = [(Fraction(int(S[i][0])), Fraction(int(S[i][1])),
                                                 Fraction(float(np.float32(S[i][2])))) for i in t]
    det = (u1 - u0) * (v2 - v0) - (u2 - u0) * (v1 - v0)
    A = ((d1 - d0) * (v2 - v0) - (d2 - d0) * (v1 - v0)) / det
    B = ((u1 - u0) * (d2 - d0) - (u2 - u0) * (d1 - d0)) / det
    C = d0 - A * u0 - B * v0
    return A, B, C


def _random_supports(seed, n, W, H, integer_d=False):
    rng = np.random.default_rng(seed)
    pts = {(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(n)}
    S = []
    for (u, v) in pts:
        d = float(rng.integers(0, 128)) if integer_d else float(np.float32(rng.uniform(0, 128)))
        S.append((u, v, d))
    return S


@pytest.mark.parametrize("seed", range(4))
def test_plane_passes_through_its_three_supports(seed):
    W, H = 120, 90
    S = _random_supports(seed, 80, W, H)
    tris = oracle.triangulate(S, W)
    for t in tris:
        A, B, C = _exact_plane(S, t)
        for i in t:   # the exact plane passes through each support disparity
            assert A * int(S[i][0]) + B * int(S[i][1]) + C == Fraction(float(np.float32(S[i][2])))
        a, b, d0, u0, v0 = oracle.plane_of(S, t)
        # float32 anchor form: exact at the anchor, within 1e-4 px at the other vertices
        assert d0 == np.float32(S[t[0]][2]) and (u0, v0) == (S[t[0]][0], S[t[0]][1])
        for i in t[1:]:
            du, dv = int(S[i][0]) - u0, int(S[i][1]) - v0
            val = (d0 + a * np.float32(du)) + b * np.float32(dv)
            assert abs(float(val) - S[i][2]) <= 1e-4 * max(1.0, abs(du) + abs(dv)) / 8 + 1e-4
        # slope equals numpy's linear solve of [u v 1] pi = d
        M = np.array([[S[i][0], S[i][1], 1.0] for i in t])
        pi = np.linalg.solve(M, np.array([S[i][2] for i in t], dtype=np.float64))
        assert abs(float(a) - pi[0]) <= 1e-6 * max(1.0, abs(pi[0]))
        assert abs(float(b) - pi[1]) <= 1e-6 * max(1.0, abs(pi[1]))
        assert abs(float(a) - float(A)) <= 1e-6 * max(1.0, abs(float(A)))


def _brute_owner(S, tris, W, H):
    """Per pixel, test every triangle with the perturbed point (u + e, v + e^2) for a
    concrete small rational e (independent of the oracle's edge rule)."""
    e = Fraction(1, 10**6)
    owner = -np.ones((H, W), dtype=np.int64)
    count = np.zeros((H, W), dtype=np.int64)
    P = [(int(s[0]), int(s[1])) for s in S]
    for k, t in enumerate(tris):
        xs = [P[i][0] for i in t]
        ys = [P[i][1] for i in t]
        for v in range(max(0, min(ys) - 1), min(H, max(ys) + 2)):
            for u in range(max(0, min(xs) - 1), min(W, max(xs) + 2)):
                px, py = u + e, v + e * e
                inside = True
                for j in range(3):
                    ax, ay = P[t[j]]
                    bx, by = P[t[(j + 1) % 3]]
                    if (bx - ax) * (py - ay) - (by - ay) * (px - ax) <= 0:
                        inside = False
                        break
                if inside:
                    owner[v, u] = k
                    count[v, u] += 1
    return owner, count


def _in_hull_perturbed(S, W, H):
    from scipy.spatial import ConvexHull
    P = np.array([(s[0], s[1]) for s in S], dtype=np.float64)
    hull = ConvexHull(P)
    e = 1e-6
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    inside = np.ones((H, W), dtype=bool)
    for eq in hull.equations:            # n . x + c <= 0 inside
        inside &= eq[0] * (uu + e) + eq[1] * (vv + e * e) + eq[2] < 0
    return inside


@pytest.mark.parametrize("seed,grid", [(0, False), (1, True), (2, False)])
def test_every_hull_pixel_has_exactly_one_owner(seed, grid):
    W, H = 48, 36
    if grid:   # cocircular grid: every pixel on a diagonal or grid line is a tie case
        S = [(5 + 6 * i, 3 + 6 * j, float(i + j)) for j in range(6) for i in range(7)]
    else:
        S = _random_supports(seed, 30, W, H)
    tris = oracle.triangulate(S, W)
    owner, count = _brute_owner(S, tris, W, H)
    assert count.max() <= 1
    D = oracle.interpolate(S, tris, W, H)
    assert (np.isfinite(D) == (count == 1)).all()
    assert ((count == 1) == _in_hull_perturbed(S, W, H)).all()
    for k, t in enumerate(tris):
        us, vs = owned_pixels(S, t, W, H)
        assert (owner[vs, us] == k).all() and len(us) == (owner == k).sum()


@pytest.mark.parametrize("seed", range(3))
def test_interpolation_stays_within_vertex_range(seed):
    W, H = 100, 80
    S = _random_supports(seed, 60, W, H)
    tris = oracle.triangulate(S, W)
    D = oracle.interpolate(S, tris, W, H)
    for t in tris:
        us, vs = owned_pixels(S, t, W, H)
        ds = [S[i][2] for i in t]
        vals = D[vs, us]
        assert (vals >= min(ds) - 1e-4).all() and (vals <= max(ds) + 1e-4).all()
        A, B, C = _exact_plane(S, t)
        for u, v, x in list(zip(us, vs, vals))[:20]:
            assert abs(float(A * int(u) + B * int(v) + C) - float(x)) <= 1e-3


def test_single_plane_exact_recovery_from_true_supports():
    """Supports on the nodes of the 10 px grid, taking the true integer disparity of a
    single slanted plane: the interpolation reproduces the plane everywhere inside the
    hull to within 1e-3 px."""
    W, H, g = 160, 120, 10
    sc = scenes.slanted_plane(W, H, d0=20, p=1, q=-1, g=g)
    S = [(u, v, float(sc.disp[v, u])) for v in range(g // 2, H, g) for u in range(g // 2, W, g)]
    assert all(s[2] == round(s[2]) for s in S)
    D = oracle.interpolate(S, oracle.triangulate(S, W), W, H)
    m = np.isfinite(D)
    assert m.sum() > 0.8 * W * H
    assert np.abs(D[m] - sc.disp[m]).max() <= 1e-3


def test_single_plane_exact_recovery_end_to_end():
    """Single slanted plane, no noise, through the whole first iteration: on every
    triangle whose three matched supports carry the true disparity, D_it equals the
    true disparity within 1e-3 px (a slanted surface shears the census window, so a
    support can be a pixel off; those triangles are excluded and must be few)."""
    W, H, g = 200, 150, 10
    sc = scenes.slanted_plane(W, H, d0=24, p=1, q=1, g=g, seed=3)
    p = oracle.Params(d_min=0, d_max=63, census_w=7, census_h=7, t_hi=10, t_lo=5,
                      grad_thr=16, n_iters=1, uniqueness=3)
    r = oracle.solve(sc.left, sc.right, p, trace=True)
    S = r["iters"][0]["S"]
    tris = r["iters"][0]["tris"]
    D = r["iters"][0]["D_it"]
    exact = [s[2] == sc.disp[s[1], s[0]] for s in S]
    assert sum(exact) >= 0.9 * len(S) and len(S) > 150
    good = [t for t in tris if all(exact[i] for i in t)]
    assert len(good) >= 0.7 * len(tris)
    for t in good:
        us, vs = owned_pixels(S, t, W, H)
        assert np.abs(D[vs, us] - sc.disp[vs, us]).max(initial=0.0) <= 1e-3


def test_no_triangles_means_all_nan():
    D = oracle.interpolate([(1, 1, 3.0), (5, 5, 3.0)], [], 8, 8)
    assert np.isnan(D).all()
