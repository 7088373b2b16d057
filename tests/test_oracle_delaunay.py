"""Pins of the oracle's Delaunay triangulation (exact predicates, perturbed ties)."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.delaunay import delaunay_points

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _lifted_sign(a, b, c, d, prio):
    """Perturbed in-circle sign computed a second, independent way: evaluate the 4x4
    lifted determinant with z_i = u^2 + v^2 + eps^(rank_i) for a concrete tiny eps
    (exact rationals), shrinking eps until the sign stabilises. rank 0 = highest
    priority = largest eps."""
    pts = [a, b, c, d]
    ranks = {i: r for r, i in enumerate(sorted(range(4), key=lambda k: prio[k]))}
    last = None
    for e in (Fraction(1, 10**3), Fraction(1, 10**6), Fraction(1, 10**12)):
        rows = [[Fraction(p[0]), Fraction(p[1]), Fraction(p[0] ** 2 + p[1] ** 2) + e ** (ranks[i] + 1),
                 Fraction(1)] for i, p in enumerate(pts)]
        det = _det4(rows)
        s = (det > 0) - (det < 0)
        if last is not None and s == last and s != 0:
            return s
        last = s
    return last


def _det4(m):
    def det3(a):
        return (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
                - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
                + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))
    tot = 0
    for j in range(4):
        minor = [row[:j] + row[j + 1:] for row in m[1:]]
        tot += (-1) ** j * m[0][j] * det3(minor)
    return tot


def _brute_triangles(pts, W):
    """Every counter-clockwise triple whose perturbed circumcircle is empty."""
    prio = [v * W + u for (u, v) in pts]
    out = set()
    n = len(pts)
    for i, j, k in itertools.combinations(range(n), 3):
        o = _orient(pts[i], pts[j], pts[k])
        if o == 0:
            continue
        t = (i, j, k) if o > 0 else (i, k, j)
        ok = True
        for m in range(n):
            if m in t:
                continue
            s = _lifted_sign(pts[t[0]], pts[t[1]], pts[t[2]], pts[m],
                             (prio[t[0]], prio[t[1]], prio[t[2]], prio[m]))
            if s > 0:
                ok = False
                break
        if ok:
            out.add(frozenset(t))
    return out


def _as_sets(tris):
    return {frozenset(t) for t in tris}


def _hull_count_and_area2(pts):
    """Points on the convex hull boundary (collinear ones included) and twice its area,
    by brute force: a point is on the boundary iff some supporting line through two
    points has every point on one side and contains it."""
    n = len(pts)
    on = set()
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            side = [_orient(pts[i], pts[j], p) for p in pts]
            if all(s >= 0 for s in side):
                for k in range(n):
                    if side[k] == 0:
                        on.add(k)
    # twice the area via the hull polygon of extreme points (gift wrapping on boundary)
    bpts = sorted({pts[k] for k in on})
    cx = sum(p[0] for p in bpts) / len(bpts)
    cy = sum(p[1] for p in bpts) / len(bpts)
    bpts.sort(key=lambda p: np.arctan2(p[1] - cy, p[0] - cx))
    area2 = 0
    for a, b in zip(bpts, bpts[1:] + bpts[:1]):
        area2 += a[0] * b[1] - a[1] * b[0]
    return len(on), abs(area2)


def _check_triangulation(pts, tris):
    n = len(pts)
    h, area2 = _hull_count_and_area2(pts)
    assert len(tris) == 2 * n - 2 - h                       # Euler count
    assert sum(_orient(*(pts[i] for i in t)) for t in tris) == area2
    for t in tris:
        assert _orient(pts[t[0]], pts[t[1]], pts[t[2]]) > 0
    used = {i for t in tris for i in t}
    assert used == set(range(n))                            # every point is a vertex


def _read_square():
    W = None
    pts, tris = [], []
    for line in open(os.path.join(GOLDEN, "delaunay_unit_square.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        vals = [int(v) for v in vals]
        if key == "W":
            W = vals[0]
        elif key == "points":
            pts = list(zip(vals[0::2], vals[1::2]))
        elif key == "tri":
            tris.append(frozenset(zip(vals[0::2], vals[1::2])))
    return W, pts, tris


def test_unit_square_hand_derived_tie():
    W, pts, expected = _read_square()
    for perm in itertools.permutations(range(4)):
        P = [pts[i] for i in perm]
        got = {frozenset(P[i] for i in t) for t in delaunay_points(P, W)}
        assert got == set(expected)


@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (8, 6)])
def test_regular_grid_uses_antidiagonals(nx, ny):
    """Every grid square is split by the diagonal that avoids its top-left corner
    (the corner with the smallest raster index gets the largest lift)."""
    g = 10
    pts = [(5 + i * g, 5 + j * g) for j in range(ny) for i in range(nx)]
    W = 5 + nx * g
    got = {frozenset(pts[i] for i in t) for t in delaunay_points(pts, W)}
    exp = set()
    for j in range(ny - 1):
        for i in range(nx - 1):
            tl, tr = (5 + i * g, 5 + j * g), (5 + (i + 1) * g, 5 + j * g)
            bl, br = (5 + i * g, 5 + (j + 1) * g), (5 + (i + 1) * g, 5 + (j + 1) * g)
            exp.add(frozenset((tl, tr, bl)))
            exp.add(frozenset((tr, br, bl)))
    assert got == exp


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_small_sets(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 11))
    span = 4 if seed % 2 == 0 else 40        # small span -> many collinear / cocircular ties
    pts = list({(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)})
    rng.shuffle(pts)
    W = 64
    if len(pts) < 3 or all(_orient(pts[0], pts[1], p) == 0 for p in pts):
        return
    got = _as_sets(delaunay_points(pts, W))
    assert got == _brute_triangles(pts, W)
    _check_triangulation(pts, delaunay_points(pts, W))


def test_sos_sign_matches_concrete_perturbation():
    rng = np.random.default_rng(7)
    for _ in range(300):
        P = [(int(rng.integers(0, 4)), int(rng.integers(0, 4))) for _ in range(4)]
        if len(set(P)) < 4 or _orient(P[0], P[1], P[2]) == 0:
            continue
        prio = [v * 8 + u for (u, v) in P]
        assert oracle.incircle_sos(*P, prio) == _lifted_sign(*P, prio)


@pytest.mark.parametrize("seed,n,span", [(0, 200, 60), (1, 300, 2000), (2, 150, 25)])
def test_empty_circumcircle_and_counts(seed, n, span):
    rng = np.random.default_rng(seed)
    pts = list({(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)})
    W = span
    tris = delaunay_points(pts, W)
    _check_triangulation(pts, tris)
    prio = [v * W + u for (u, v) in pts]
    for t in tris:
        a, b, c = (pts[i] for i in t)
        for m in range(len(pts)):
            if m in t:
                continue
            assert oracle.incircle_sos(a, b, c, pts[m], (prio[t[0]], prio[t[1]], prio[t[2]], prio[m])) < 0


def test_general_position_equals_qhull():
    scipy_spatial = pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(11)
    pts = list({(int(rng.integers(0, 8000)), int(rng.integers(0, 8000))) for _ in range(400)})
    # require general position: no in-circle test of the final mesh is a tie
    tris = delaunay_points(pts, 8192)
    q = scipy_spatial.Delaunay(np.array(pts, dtype=np.float64))
    assert _as_sets(tris) == {frozenset(int(i) for i in s) for s in q.simplices}


def test_insertion_order_independent_and_duplicates():
    rng = np.random.default_rng(5)
    base = [(int(rng.integers(0, 30)), int(rng.integers(0, 30))) for _ in range(60)]
    S = [(u, v, 1.0) for (u, v) in base]
    ref = {frozenset(S[i][:2] for i in t) for t in oracle.triangulate(S, 30)}
    for s in range(3):
        perm = list(rng.permutation(len(S)))
        S2 = [S[i] for i in perm]
        got = {frozenset(S2[i][:2] for i in t) for t in oracle.triangulate(S2, 30)}
        assert got == ref
    # duplicates refer to the first occurrence
    tris = oracle.triangulate(S, 30)
    firsts = {}
    for i, s in enumerate(S):
        firsts.setdefault(s[:2], i)
    assert all(i == firsts[S[i][:2]] for t in tris for i in t)


def test_degenerate_inputs():
    assert oracle.triangulate([], 10) == []
    assert oracle.triangulate([(1, 1, 0.0), (2, 2, 0.0)], 10) == []
    assert oracle.triangulate([(i, 2 * i, 0.0) for i in range(6)], 20) == []
    # collinear run plus one point: a fan of triangles, every point used
    S = [(i, 0, 0.0) for i in range(6)] + [(2, 5, 0.0)]
    tris = oracle.triangulate(S, 10)
    assert len(tris) == 5
    with pytest.raises(ValueError):
        oracle.triangulate([(9000, 0, 0.0), (0, 1, 0.0), (1, 0, 0.0)], 9001)


def test_canonical_form():
    rng = np.random.default_rng(2)
    S = [(int(rng.integers(0, 50)), int(rng.integers(0, 50)), 0.0) for _ in range(40)]
    tris = oracle.triangulate(S, 50)
    assert tris == sorted(tris)
    for t in tris:
        keys = [(S[i][1], S[i][0]) for i in t]
        assert keys[0] == min(keys)
        assert _orient(S[t[0]], S[t[1]], S[t[2]]) > 0
