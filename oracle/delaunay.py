"""Delaunay triangulation of the support points. Test infrastructure only.

Sec. III-A builds the piecewise-planar mesh G(S) by Delaunay triangulation of the
support pixels. The paper does not say how ties are broken; support pixels on a
regular grid make every grid square cocircular, so the reading used here is:

* exact integer predicates (coordinates in [0, 8191], so every determinant below
  fits in a signed 64-bit integer);
* cocircular ties resolved by Simulation of Simplicity (Edelsbrunner and Muecke,
  1990) applied to the lifting z = u^2 + v^2 + eps_i, where a point with a smaller
  raster index v*W + u gets the (infinitely) larger eps. The sign of a zero in-circle
  determinant is then the sign of the cofactor of the highest-priority point whose
  cofactor is non-zero;
* duplicate pixels are dropped, the first occurrence kept.

The result is the unique triangulation of the perturbed point set; it contains
every distinct input point, including points on the hull's straight runs.

The construction is Bowyer-Watson insertion written from its definition: every
triangle whose (perturbed) circumcircle strictly contains the new point is
removed, and the new point is joined to each edge of the hole's boundary. Hull
edges carry "ghost" triangles whose circumcircle is the open outer half-plane of
the edge plus the open edge itself. Conflicts are found by testing every triangle
(no point location), which is slow but plainly correct.
"""
from typing import List, Sequence, Tuple

import numpy as np

GHOST = -1
COORD_MAX = 8191


def orient(a, b, c) -> int:
    """Twice the signed area of (a, b, c); > 0 when a, b, c turn counter-clockwise."""
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def incircle(a, b, c, d) -> int:
    """det[[x, y, x^2 + y^2, 1]] over rows a, b, c, d: > 0 when d lies strictly inside
    the circle through a, b, c (a, b, c counter-clockwise)."""
    adx, ady = a[0] - d[0], a[1] - d[1]
    bdx, bdy = b[0] - d[0], b[1] - d[1]
    cdx, cdy = c[0] - d[0], c[1] - d[1]
    al = adx * adx + ady * ady
    bl = bdx * bdx + bdy * bdy
    cl = cdx * cdx + cdy * cdy
    return adx * (bdy * cl - cdy * bl) - ady * (bdx * cl - cdx * bl) + al * (bdx * cdy - cdx * bdy)


def incircle_sos(a, b, c, d, prio: Sequence[int]) -> int:
    """Sign (+1 / -1, never 0) of the in-circle determinant under the perturbation
    z_i += eps_i, eps larger for smaller ``prio`` (raster index)."""
    det = incircle(a, b, c, d)
    if det != 0:
        return 1 if det > 0 else -1
    # d(det)/d(z_i): cofactor of the lifted column in row i of rows (a, b, c, d)
    cof = [orient(b, c, d), -orient(a, c, d), orient(a, b, d), -orient(a, b, c)]
    for i in sorted(range(4), key=lambda k: prio[k]):
        if cof[i] != 0:
            return 1 if cof[i] > 0 else -1
    raise AssertionError("degenerate in-circle test on collinear points")


def _ghost_conflict(a, b, p) -> bool:
    """Hull edge a->b (interior on its left): p lies strictly on the outer side, or on
    the open segment (a, b)."""
    o = orient(a, b, p)
    if o < 0:
        return True
    if o > 0:
        return False
    dot1 = (p[0] - a[0]) * (b[0] - a[0]) + (p[1] - a[1]) * (b[1] - a[1])
    dot2 = (p[0] - b[0]) * (a[0] - b[0]) + (p[1] - b[1]) * (a[1] - b[1])
    return dot1 > 0 and dot2 > 0


def _canonical(t, pts):
    """Rotate a counter-clockwise triangle so its first vertex has the smallest (v, u)."""
    k = min(range(3), key=lambda i: (pts[t[i]][1], pts[t[i]][0]))
    return (t[k], t[(k + 1) % 3], t[(k + 2) % 3])


def delaunay_points(pts: List[Tuple[int, int]], W: int) -> List[Tuple[int, int, int]]:
    """Triangles (indices into ``pts``, all distinct) of the perturbed Delaunay
    triangulation, counter-clockwise, first vertex = smallest (v, u), sorted."""
    n = len(pts)
    for (u, v) in pts:
        if not (0 <= u <= COORD_MAX and 0 <= v <= COORD_MAX):
            raise ValueError("coordinates must lie in [0, 8191]")
    if n < 3:
        return []
    prio = [v * W + u for (u, v) in pts]
    X = np.array([p[0] for p in pts], dtype=np.int64)
    Y = np.array([p[1] for p in pts], dtype=np.int64)
    # first triangle: points 0, 1 and the first point not collinear with them
    k0 = next((k for k in range(2, n) if orient(pts[0], pts[1], pts[k]) != 0), None)
    if k0 is None:
        return []
    first = (0, 1, k0) if orient(pts[0], pts[1], pts[k0]) > 0 else (0, k0, 1)
    # solid triangles (counter-clockwise) and hull edges a->b with the interior on the left
    tri = np.array([first], dtype=np.int64)
    hull = np.array([(first[0], first[1]), (first[1], first[2]), (first[2], first[0])],
                    dtype=np.int64)
    for q in range(2, n):
        if q == k0:
            continue
        px, py = int(X[q]), int(Y[q])
        # --- solid triangles in conflict: exact in-circle, perturbed on ties
        A, B, C = tri[:, 0], tri[:, 1], tri[:, 2]
        adx, ady = X[A] - px, Y[A] - py
        bdx, bdy = X[B] - px, Y[B] - py
        cdx, cdy = X[C] - px, Y[C] - py
        al = adx * adx + ady * ady
        bl = bdx * bdx + bdy * bdy
        cl = cdx * cdx + cdy * cdy
        det = adx * (bdy * cl - cdy * bl) - ady * (bdx * cl - cdx * bl) + al * (bdx * cdy - cdx * bdy)
        conflict = det > 0
        for t in np.nonzero(det == 0)[0]:
            a, b, c = (int(v) for v in tri[t])
            s = incircle_sos(pts[a], pts[b], pts[c], pts[q], (prio[a], prio[b], prio[c], prio[q]))
            conflict[t] = s > 0
        # --- ghost triangles in conflict
        # (vectorised form of _ghost_conflict over every hull edge)
        HA, HB = hull[:, 0], hull[:, 1]
        o = (X[HB] - X[HA]) * (py - Y[HA]) - (Y[HB] - Y[HA]) * (px - X[HA])
        dot1 = (px - X[HA]) * (X[HB] - X[HA]) + (py - Y[HA]) * (Y[HB] - Y[HA])
        dot2 = (px - X[HB]) * (X[HA] - X[HB]) + (py - Y[HB]) * (Y[HA] - Y[HB])
        gconf = (o < 0) | ((o == 0) & (dot1 > 0) & (dot2 > 0))
        # --- boundary of the hole: directed edges whose reverse is not in the hole
        edges = set()
        for (a, b, c) in tri[conflict]:
            edges.update({(int(a), int(b)), (int(b), int(c)), (int(c), int(a))})
        for (a, b) in hull[gconf]:
            a, b = int(a), int(b)
            edges.update({(b, a), (a, GHOST), (GHOST, b)})  # ghost triangle (b, a, ghost)
        boundary = [e for e in edges if (e[1], e[0]) not in edges]
        assert boundary, "point in conflict with nothing"
        new_tri, new_hull = [], []
        for (x, y) in boundary:
            if x != GHOST and y != GHOST:
                assert orient(pts[x], pts[y], pts[q]) > 0
                new_tri.append((x, y, q))
            elif y == GHOST:       # ghost triangle (x, ghost, q): hull edge x -> q
                new_hull.append((x, q))
            else:                  # ghost triangle (ghost, y, q): hull edge q -> y
                new_hull.append((q, y))
        tri = np.concatenate([tri[~conflict], np.array(new_tri, dtype=np.int64).reshape(-1, 3)])
        hull = np.concatenate([hull[~gconf], np.array(new_hull, dtype=np.int64).reshape(-1, 2)])
    out = [_canonical(tuple(int(v) for v in t), pts) for t in tri]
    return sorted(out)


def triangulate(S: Sequence, W: int) -> List[Tuple[int, int, int]]:
    """Delaunay triangles of supports ``S`` (tuples starting with u, v). Indices refer
    to ``S``; a duplicated pixel is represented by its first occurrence."""
    first = {}
    keep = []
    for i, s in enumerate(S):
        key = (int(s[0]), int(s[1]))
        if key not in first:
            first[key] = i
            keep.append(i)
    pts = [(int(S[i][0]), int(S[i][1])) for i in keep]
    tris = delaunay_points(pts, W)
    out = []
    for t in tris:
        out.append(tuple(keep[j] for j in t))
    # re-canonicalise on the original indices (same vertices, same rotation rule)
    Sp = {i: (int(S[i][0]), int(S[i][1])) for i in keep}
    out = [_canonical(t, Sp) for t in out]
    return sorted(out)
